// Reduced-precision forms of the exchange build (K); J is always built in
// FP64 (it is bound by reading L).
//
//   FP32  : the half transform X^P = Lt^P C runs in FP64 and writes X rounded
//           to FP32 (k_half_sparse<HALF_F32>); the product K = sum_P X^P^T X^P
//           runs on v_mfma_f32_16x16x4f32 (k_syrk_rows_lp), FP32 accumulation
//           inside k-slabs of 32 and FP64 across slabs.
//   BF16X3: the half transform runs in FP64 and writes X split into three BF16
//           planes (k_half_sparse<true>); the product K reads the planes
//           (k_syrk_bf16x3).  Every operand x is split as x = b0 + b1 + b2
//           (round-to-nearest BF16 each: b0 = bf16(x), b1 = bf16(x - b0),
//           b2 = bf16(x - b0 - b1)), and a product a*c keeps the six terms up
//           to order 2^-16: a0c0 + a0c1 + a1c0 + a0c2 + a1c1 + a2c0 (Henry, Tang
//           & Heinecke, "Leveraging the bfloat16 artificial intelligence
//           datatype for higher-precision computations", ARITH 2019), on
//           v_mfma_f32_16x16x32_bf16, FP32 inside steps of 32 and FP64 across.
//
// Result lane layout of both FP32-accumulating instructions (read back on
// gfx950): lane l, element v holds D[m = 4 (l / 16) + v][n = l % 16].
// Operands: FP32 16x16x4 as the FP64 one (A[m = l%16][k = l/16]); BF16
// 16x16x32 lane l holds 8 consecutive k = 8 (l / 16) + j of row/column l % 16.
#include "cd_device.hpp"
#include "cd_mfma.hpp"

namespace cdk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum LpMode { LP_F32 = 1 };

constexpr int LP_TKC = 32;     // k-chunk staged in LDS
constexpr int LP_SLAB = 32;    // FP32 accumulation length before folding into FP64

__device__ __forceinline__ int lp_row(int lane, int v) { return 4 * (lane >> 4) + v; }

// LDS staging of one k-chunk of FP32 operands for a 64 x 64 tile:
//   k-major sources   sA32[k][m], sB32[k][n]
//   k-contiguous (KC) sA32[m][k], sB32[n][k]  (rows padded to TKC + 1)
// so that the LDS writes follow the contiguous index of the global loads.
template <int MODE, bool KC = false>
struct LpStage {
    static_assert(MODE == LP_F32, "FP32 staging only");
    static constexpr int kF32Ld = LP_TKC + 1;    // padded row (KC)
    static constexpr int kBytes = 2 * 64 * (LP_TKC + 1) * 4;
    __device__ static __forceinline__ int f32_index(int k, int m)
    {
        return KC ? m * kF32Ld + k : k * 64 + m;
    }
    static constexpr int kPer = LP_TKC * 64 / 256;   // elements per thread per operand

    // element e of a chunk -> (k, m), following the operand's contiguous index:
    // m fastest for k-major sources, k fastest for k-contiguous ones (KC)
    __device__ static __forceinline__ void coord(int e, int &k, int &m)
    {
        if (KC) {
            m = e / LP_TKC;
            k = e % LP_TKC;
        } else {
            k = e >> 6;
            m = e & 63;
        }
    }
    template <class LA, class LB>
    __device__ static __forceinline__ void fetch(LA la, LB lb, int64_t k0, int64_t kend,
                                                 double (&ra)[kPer], double (&rb)[kPer])
    {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = threadIdx.x + 256 * u;
            int k, m;
            coord(e, k, m);
            const bool ok = k0 + k < kend;
            const int64_t kk = ok ? k0 + k : kend - 1;   // always valid: load, then select
            const double va = la(kk, m), vb = lb(kk, m);
            ra[u] = ok ? va : 0.0;
            rb[u] = ok ? vb : 0.0;
        }
    }
    __device__ static __forceinline__ void put(unsigned char *smem, const double (&ra)[kPer],
                                               const double (&rb)[kPer])
    {
        float *sA = reinterpret_cast<float *>(smem);
        float *sB = sA + 64 * kF32Ld;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            int k, m;
            coord(threadIdx.x + 256 * u, k, m);
            sA[f32_index(k, m)] = (float)ra[u];
            sB[f32_index(k, m)] = (float)rb[u];
        }
    }
    // multiply the staged chunk into acc[r] (rows 16 r.., columns 16 w..)
    __device__ static __forceinline__ void mma(const unsigned char *smem, f32x4 (&acc)[4])
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const float *sA = reinterpret_cast<const float *>(smem);
        const float *sB = sA + 64 * kF32Ld;
#pragma unroll
        for (int ks = 0; ks < LP_TKC; ks += 4) {
            const int kk = ks + (lane >> 4);
            const float b = sB[f32_index(kk, 16 * w + (lane & 15))];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float a = sA[f32_index(kk, 16 * r + (lane & 15))];
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[r], 0, 0, 0);
            }
        }
    }
};

// acc64[r][v] += sum_k A(k, m) B(k, n) over [kbeg, kend), FP32 inside slabs.
template <int MODE, bool KC, class LA, class LB>
__device__ __forceinline__ void lp_tile(int64_t kbeg, int64_t kend, LA la, LB lb,
                                        double (&acc64)[4][4], unsigned char *smem)
{
    using S = LpStage<MODE, KC>;
    f32x4 acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (kbeg >= kend) return;
    double ra[S::kPer], rb[S::kPer];
    S::fetch(la, lb, kbeg, kend, ra, rb);
    int in_slab = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += LP_TKC) {
        S::put(smem, ra, rb);
        __syncthreads();
        if (k0 + LP_TKC < kend) S::fetch(la, lb, k0 + LP_TKC, kend, ra, rb);
        S::mma(smem, acc);
        __syncthreads();
        in_slab += LP_TKC;
        if (in_slab >= LP_SLAB || k0 + LP_TKC >= kend) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    acc64[r][v] += (double)acc[r][v];
                    acc[r][v] = 0.f;
                }
            in_slab = 0;
        }
    }
}

// Partial K from row-major FP32 X, reduced precision:
//   Kp[s][mu][nu] = sum_{k in slab s} X[mu][k] X[nu][k]   (lower tile pairs)
template <int MODE>
__global__ __launch_bounds__(256) void k_syrk_rows_lp(const float *__restrict__ X, int64_t ldx,
                                                      int N, const int64_t *__restrict__ n_vectors,
                                                      int ncol, int nsplit,
                                                      double *__restrict__ Kp)
{
    __shared__ __align__(16) unsigned char smem[LpStage<MODE, true>::kBytes];
    int t, s;
    syrk_tile_split(N, nsplit, t, s);
    int tm = 0;
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    const int tn = t - tm * (tm + 1) / 2;
    const int64_t nk = *n_vectors * ncol;
    int64_t per = (nk + nsplit - 1) / nsplit;
    per = (per + LP_SLAB - 1) / LP_SLAB * LP_SLAB;
    const int64_t kb = s * per;
    const int64_t ke = (kb + per < nk) ? kb + per : nk;
    const int m0 = tm * 64, n0 = tn * 64;
    double acc[4][4] = {};
    lp_tile<MODE, true>(
        kb, ke,
        [&](int64_t k, int m) -> double { return (double)X[min(m0 + m, N - 1) * ldx + k]; },
        [&](int64_t k, int n) -> double { return (double)X[min(n0 + n, N - 1) * ldx + k]; },
        acc, smem);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double *out = Kp + (int64_t)s * N * N;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = m0 + 16 * r + lp_row(lane, v), n = n0 + 16 * w + (lane & 15);
            if (m < N && n < N) out[(int64_t)m * N + n] = acc[r][v];
        }
}

// ---------------------------------------------------------------- 3 x BF16, large tiles
// Partial K from the three BF16 planes of X with 128 x 128 output tiles:
//   Kp[s][mu][nu] = sum_{k in split s} X[mu][k] X[nu][k]   (lower tile pairs)
// with the six products of the 3 x BF16 split (see the top of this file).
// Each wave owns a 64 x 64 quarter of the tile (4 x 4 accumulators of the
// 16x16x32 BF16 instruction), so every operand fragment read from LDS feeds
// four tiles.  A step stages 32 values of the 256 rows (the 128 rows of each
// side, all three planes: 48 KB) in one of three LDS buffers.  The loads go
// from memory straight into LDS (global_load_lds, 16 bytes per lane, a wave's
// 64 pieces filling one contiguous KB) two steps ahead of the products, so no
// registers hold them and 96 KB per compute unit are in flight; one barrier per
// step.  LDS rows are 64 bytes with no padding; the 16-byte k-group g of row r
// sits at group g ^ ((r / 4) % 4), so the 16 rows read by one quarter-wave at
// one k-group fall on 16 different 16-byte bank groups.
//
// FP32 accumulation runs over one step (32 values; each step's products start
// from a zero accumulator) and each row tile's step sums are added in FP64
// while the next row tile's products run.  Longer FP32 slabs were measured:
// with 512 values per slab the error of K grew about twentyfold (to 6e-7 Eh on
// the 1200-function workload, and 5e-6 Eh in E2), roughly in proportion to the
// slab length, so the matrix unit's FP32 accumulation rounds with a bias and
// slabs stay at one step.
//
// X holds its three planes 'plane' values apart, each of ldx-value rows padded
// to a whole number of 128-row tiles (the rows past N are never written and
// only enter K entries past N, which are not stored).
//
// Grid (one workgroup per compute unit at 144 KB of LDS): workgroup g runs on
// XCD g % 8; its j = g / 8 -th item is tile pair j % pairs of split
// 8 (j / pairs) + g % 8, so each XCD works on its own k-ranges of X and the
// tile pairs of one k-range, dispatched together, share it through that XCD's
// L2.  'nsplit' / 8 k-ranges per XCD are chosen on the host so that the
// workgroups fill an XCD's compute units in whole rounds.
constexpr int BX_TILE = 128;
constexpr int BX_TK = 32;                        // k per stage: one 16x16x32 step
constexpr int BX_ROWS = 2 * BX_TILE;             // A rows, then B rows
constexpr int BX_STAGE = 3 * BX_ROWS * BX_TK;    // bf16 elements per stage (48 KB)
constexpr int BX_LOADS = BX_STAGE * 2 / 16 / 256;   // 16-byte pieces per thread per stage (12)

// bf16 offset in a stage of k-group g (8 values) of row r of plane p
__device__ __forceinline__ int bx_off(int p, int r, int g)
{
    return 8 * ((p * BX_ROWS + r) * 4 + (g ^ ((r >> 2) & 3)));
}

__device__ __forceinline__ void bx_item(int pairs, int &tm, int &tn, int &split)
{
    const int g = blockIdx.x, xcd = g & 7, j = g >> 3;
    const int t = j % pairs;
    split = 8 * (j / pairs) + xcd;
    int m = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (m * (m + 1) / 2 > t) --m;
    while ((m + 1) * (m + 2) / 2 <= t) ++m;
    tm = m;
    tn = t - m * (m + 1) / 2;
}

__global__ __launch_bounds__(256) void k_syrk_bf16x3(const __bf16 *__restrict__ Xp, int64_t ldx,
                                                     int64_t plane, int N,
                                                     const int64_t *__restrict__ n_vectors,
                                                     int ncol, int pairs, int nsplit,
                                                     double *__restrict__ Kp)
{
    __shared__ __align__(16) __bf16 sX0[BX_STAGE];
    __shared__ __align__(16) __bf16 sX1[BX_STAGE];
    __shared__ __align__(16) __bf16 sX2[BX_STAGE];
    int tm, tn, s;
    bx_item(pairs, tm, tn, s);
    const int64_t nk = *n_vectors * ncol;
    int64_t per = (nk + nsplit - 1) / nsplit;
    per = (per + BX_TK - 1) / BX_TK * BX_TK;
    const int64_t kb = s * per;
    const int64_t ke = (kb + per < nk) ? kb + per : nk;
    const int m0 = tm * BX_TILE, n0 = tn * BX_TILE;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;

    // Piece v of this lane is the LDS piece q = 64 (4 v + w) + lane of a stage:
    // plane (4 v + w) / 16, row 16 ((4 v + w) % 16) + lane / 4, stored k-group
    // lane % 4, which holds k-group g = (lane % 4) ^ ((lane / 16) % 4) of that
    // row.  Rows 0..127 are the A side (rows m0..), 128..255 the B side (n0..);
    // the planes hold whole 128-row tiles (rows past N are padding), so a
    // piece's address is this lane's offset plus a wave-uniform one.
    const int g = (lane & 3) ^ ((lane >> 4) & 3);
    const __bf16 *lane_src = Xp + (int64_t)(lane >> 2) * ldx + 8 * g;
    auto wave_off = [&](int v) __attribute__((always_inline)) -> int64_t {
        const int b = 4 * v + w, rb = b & 15;
        const int row0 = (rb < 8) ? m0 + 16 * rb : n0 + 16 * (rb - 8);
        return (int64_t)(b >> 4) * plane + (int64_t)row0 * ldx;
    };
    // a full step straight into LDS (12 loads per lane); a partial last step
    // through registers with the values past ke set to zero
    auto load_step = [&](__bf16 *stage, int64_t k0) __attribute__((always_inline)) {
        if (k0 + BX_TK <= ke) {
#pragma unroll
            for (int v = 0; v < BX_LOADS; ++v)
                lds_dma16(lane_src + wave_off(v) + k0, (lds_void *)(stage + 512 * (4 * v + w)));
        } else {
#pragma unroll
            for (int v = 0; v < BX_LOADS; ++v) {
                const __bf16 *src = lane_src + wave_off(v) + k0;
                bf16x8 x;
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = (k0 + 8 * g + e < ke) ? src[e] : (__bf16)0.0f;
                *reinterpret_cast<bf16x8 *>(stage + 512 * (4 * v + w) + 8 * lane) = x;
            }
        }
    };

    double acc64[4][4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc64[i][j][e] = 0.0;
    const int lr = lane & 15, kg = lane >> 4;

    // One staged step: for each row tile i, the six products into four fresh
    // FP32 accumulators (one per column tile), then their FP64 fold.  The rows
    // are software-pipelined: the A fragments of row i + 1 are read before the
    // products of row i + 1 are issued, and the fold of row i comes after
    // them, so the vector unit adds while the matrix unit multiplies.
    // Products go smallest first: a0b2, a1b1, a0b1, a2b0, a1b0, a0b0.
    auto mma_step = [&](const __bf16 *S) __attribute__((always_inline)) {
        bf16x8 b[3][4];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[p][j] = *reinterpret_cast<const bf16x8 *>(
                    S + bx_off(p, BX_TILE + 64 * wc + 16 * j + lr, kg));
        auto read_a = [&](int i, bf16x8 (&a)[3]) __attribute__((always_inline)) {
#pragma unroll
            for (int p = 0; p < 3; ++p)
                a[p] = *reinterpret_cast<const bf16x8 *>(S + bx_off(p, 64 * wr + 16 * i + lr, kg));
        };
        auto products = [&](const bf16x8 (&a)[3], f32x4 (&t)[4]) __attribute__((always_inline)) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                t[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2][j],
                                                               f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                t[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1][j], t[j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                t[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1][j], t[j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                t[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0][j], t[j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                t[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0][j], t[j], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                t[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0][j], t[j], 0, 0, 0);
        };
        auto fold = [&](int i, const f32x4 (&t)[4]) __attribute__((always_inline)) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc64[i][j][e] += (double)t[j][e];
        };
        bf16x8 a0[3], a1[3];
        f32x4 t0[4], t1[4];
        read_a(0, a0);
        read_a(1, a1);
        products(a0, t0);
        read_a(2, a0);
        products(a1, t1);
        fold(0, t0);
        read_a(3, a1);
        products(a0, t0);
        fold(1, t1);
        products(a1, t1);
        fold(2, t0);
        fold(3, t1);
    };
    // step c: wait for its own loads (the next step's may stay in flight), a
    // barrier (every wave's pieces of step c have landed, and every wave is
    // done with the buffer that step c + 2 refills), the loads of step c + 2,
    // then the products of step c
    const int64_t nch = (ke > kb) ? (ke - kb + BX_TK - 1) / BX_TK : 0;
    auto step = [&](int64_t c, const __bf16 *cur, __bf16 *refill) __attribute__((always_inline)) {
        if (c + 1 < nch) wait_vmcnt<BX_LOADS>();
        else wait_vmcnt<0>();
        lds_barrier();
        if (c + 2 < nch) load_step(refill, kb + (c + 2) * BX_TK);
        mma_step(cur);
    };
    if (nch > 0) load_step(sX0, kb);
    if (nch > 1) load_step(sX1, kb + BX_TK);
    for (int64_t c = 0; c < nch; c += 3) {
        step(c, sX0, sX2);
        if (c + 1 < nch) step(c + 1, sX1, sX0);
        if (c + 2 < nch) step(c + 2, sX2, sX1);
    }
    double *out = Kp + (int64_t)s * N * N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + 64 * wr + 16 * i + lp_row(lane, e);
                const int n = n0 + 64 * wc + 16 * j + lr;
                if (m < N && n < N) out[(int64_t)m * N + n] = acc64[i][j][e];
            }
}

}  // namespace cdk

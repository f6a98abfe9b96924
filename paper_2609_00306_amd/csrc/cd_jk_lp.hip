// Reduced-precision forms of the exchange build (K); J is always built in
// FP64 (it is bound by reading L).
//
//   FP32  : the half transform X^P = Lt^P C runs in FP64 and writes X rounded
//           to FP32 (k_half_sparse<HALF_F32>); the product K = sum_P X^P^T X^P
//           runs on v_mfma_f32_16x16x4f32 (k_syrk_f32), FP32 accumulation
//           inside k-steps of 32 and FP64 across steps.
//   BF16X3: the half transform runs in FP64 and writes X split into three BF16
//           planes (k_half_sparse<HALF_BF16X3>); the product K reads the planes
//           (k_syrk_bf16x3).  Every operand x is split as x = b0 + b1 + b2
//           (round-to-nearest BF16 each, split_bf16x3), and a product a*c
//           keeps the six terms up to order 2^-16: a0c0 + a0c1 + a1c0 + a0c2 + a1c1 + a2c0 (Henry, Tang
//           & Heinecke, "Leveraging the bfloat16 artificial intelligence
//           datatype for higher-precision computations", ARITH 2019), on
//           v_mfma_f32_16x16x32_bf16, FP32 inside steps of 32 and FP64 across.
//
// Both read X in the k-blocked layout the half transform writes (xb_index):
// one k-step of 32 values of 128 rows is one contiguous run of memory.
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

__device__ __forceinline__ int lp_row(int lane, int v) { return 4 * (lane >> 4) + v; }

// Work item of the 3 x BF16 exchange product, launched
// as pairs x nsplit workgroups with nsplit a multiple of 8: workgroup g runs
// on XCD g % 8; its j = g / 8 -th item is tile pair j % pairs (lower
// triangle, row-major) of split 8 (j / pairs) + g % 8.
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

// ---------------------------------------------------------------- FP32
// Partial K from the k-blocked FP32 X with 64 x 64 output tiles:
//   Kp[s][mu][nu] = sum_{k in split s} X[mu][k] X[nu][k]   (lower tile pairs)
// Work items as the FP64 product (syrk_tile_split: the tile pairs of one
// k-range on one XCD).  Wave w owns the 32 x 32 quarter (rows 32 (w / 2),
// columns 32 (w % 2)) as 2 x 2 accumulators of the 16x16x4 FP32 instruction.
// A step stages 32 values of the 128 rows (both sides: 16 KB) in one of three
// LDS buffers, straight from memory (global_load_lds, 16 bytes per lane, 4
// per lane per step) two steps ahead of the products; one barrier per step.
// LDS rows are 128 bytes with no padding; the 16-byte group g of row r sits at
// g ^ ((r / 2) % 8), so the 16 rows one quarter-wave reads at one k fall on
// 16 different banks.  48 KB of LDS: three workgroups per compute unit.
// 64 x 64 tiles pad N = 1200 to 1216 rows where 128 x 128 ones pad it to 1280
// and compute more of the diagonal tiles' upper halves: 13.3 against 15.8 ms
// on the 1200-function workload.
//
// FP32 accumulation runs over one step (32 values, from zero accumulators),
// whose sums are then added in FP64.
constexpr int XF_STAGE = 128 * XB_K;                  // floats per stage (16 KB)
constexpr int XF_LOADS = XF_STAGE * 4 / 16 / 256;     // 16-byte pieces per thread per stage (4)

__global__ __launch_bounds__(256) void k_syrk_f32(const float *__restrict__ X, int64_t rows, int N,
                                                  const int64_t *__restrict__ n_vectors, int ncol,
                                                  int nsplit, double *__restrict__ Kp)
{
    __shared__ __align__(16) float sX[3 * XF_STAGE];
    int t, s;
    syrk_tile_split(N, nsplit, t, s);
    int tm = 0;
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    const int tn = t - tm * (tm + 1) / 2;
    const int64_t nk = *n_vectors * ncol;
    int64_t per = (nk + nsplit - 1) / nsplit;
    per = (per + XB_K - 1) / XB_K * XB_K;
    const int64_t kb = s * per;
    const int64_t ke = (kb + per < nk) ? kb + per : nk;
    const int m0 = tm * 64, n0 = tn * 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // piece v of this lane: LDS row r = 8 (4 v + w) + lane / 8 (rows 0..63 the
    // A side m0.., 64..127 the B side n0..; rows past N read row N - 1), slot
    // lane % 8, which holds the 16-byte group (lane % 8) ^ ((r / 2) % 8)
    int goff[XF_LOADS];
#pragma unroll
    for (int v = 0; v < XF_LOADS; ++v) {
        const int r = 8 * (4 * v + w) + (lane >> 3);
        const int grow = min((r < 64) ? m0 + r : n0 + r - 64, N - 1);
        goff[v] = grow * XB_K + 4 * ((lane & 7) ^ ((r >> 1) & 7));
    }
    // a full step straight into LDS; a partial last step through registers
    // with the values past ke set to zero
    auto load_step = [&](float *st, int64_t k0) __attribute__((always_inline)) {
        const float *base = X + (k0 / XB_K) * (rows * XB_K);
        if (k0 + XB_K <= ke) {
#pragma unroll
            for (int v = 0; v < XF_LOADS; ++v)
                lds_dma16(base + goff[v], (lds_void *)(st + 256 * (4 * v + w)));
        } else {
            for (int e = tid; e < XF_STAGE; e += 256) {
                const int r = e / XB_K, k = e % XB_K;
                const int grow = min((r < 64) ? m0 + r : n0 + r - 64, N - 1);
                st[r * XB_K + 4 * ((k >> 2) ^ ((r >> 1) & 7)) + (k & 3)] =
                    (k0 + k < ke) ? base[grow * XB_K + k] : 0.f;
            }
        }
    };
    double acc64[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc64[i][j][e] = 0.0;
    // operand of this lane at k-step q (k = 4 q + lane / 16) of a row r with
    // r % 16 = lane % 16: group q of that row, swizzled
    const int lr = lane & 15, sw = (lr >> 1) & 7, el = lane >> 4;
    const int ar = 32 * (w >> 1) + lr, br = 64 + 32 * (w & 1) + lr;
    auto mma_step = [&](const float *S) __attribute__((always_inline)) {
        f32x4 t4[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) t4[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int g = 4 * (q ^ sw) + el;
            const float a0 = S[ar * XB_K + g], a1 = S[(ar + 16) * XB_K + g];
            const float b0 = S[br * XB_K + g], b1 = S[(br + 16) * XB_K + g];
            t4[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, t4[0][0], 0, 0, 0);
            t4[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, t4[0][1], 0, 0, 0);
            t4[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, t4[1][0], 0, 0, 0);
            t4[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, t4[1][1], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc64[i][j][e] += (double)t4[i][j][e];
    };
    // step c: its own loads landed (the next step's may stay in flight), a
    // barrier (every wave's pieces of step c are in, and every wave is done
    // with the buffer that step c + 2 refills), the loads of step c + 2, then
    // the products of step c
    const int64_t nch = (ke > kb) ? (ke - kb + XB_K - 1) / XB_K : 0;
    if (nch > 0) load_step(sX, kb);
    if (nch > 1) load_step(sX + XF_STAGE, kb + XB_K);
    int buf = 0;
    for (int64_t c = 0; c < nch; ++c) {
        if (c + 1 < nch) wait_vmcnt<XF_LOADS>();
        else wait_vmcnt<0>();
        lds_barrier();
        if (c + 2 < nch) load_step(sX + ((buf == 0) ? 2 : buf - 1) * XF_STAGE, kb + (c + 2) * XB_K);
        mma_step(sX + buf * XF_STAGE);
        buf = (buf == 2) ? 0 : buf + 1;
    }
    double *out = Kp + (int64_t)s * N * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + 32 * (w >> 1) + 16 * i + lp_row(lane, e);
                const int n = n0 + 32 * (w & 1) + 16 * j + lr;
                if (m < N && n < N) out[(int64_t)m * N + n] = acc64[i][j][e];
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
// X holds its three planes 'plane' values apart, each k-blocked (xb_index)
// over 'rows' rows: N padded to a whole number of 128-row tiles (the rows past
// N are never written and only enter K entries past N, which are not stored).
//
// Grid (one workgroup per compute unit at 144 KB of LDS): workgroup g runs on
// XCD g % 8; its j = g / 8 -th item is tile pair j % pairs of split
// 8 (j / pairs) + g % 8, so each XCD works on its own k-ranges of X and the
// tile pairs of one k-range, dispatched together, share it through that XCD's
// L2.  'nsplit' / 8 k-ranges per XCD are chosen on the host so that the
// workgroups fill an XCD's compute units in whole rounds.
constexpr int BX_TILE = 128;
constexpr int BX_TK = XB_K;                   // k per stage: one 16x16x32 step, one block
constexpr int BX_ROWS = 2 * BX_TILE;             // A rows, then B rows
constexpr int BX_STAGE = 3 * BX_ROWS * BX_TK;    // bf16 elements per stage (48 KB)
constexpr int BX_LOADS = BX_STAGE * 2 / 16 / 256;   // 16-byte pieces per thread per stage (12)

// bf16 offset in a stage of k-group g (8 values) of row r of plane p
__device__ __forceinline__ int bx_off(int p, int r, int g)
{
    return 8 * ((p * BX_ROWS + r) * 4 + (g ^ ((r >> 2) & 3)));
}


__global__ __launch_bounds__(256) void k_syrk_bf16x3(const __bf16 *__restrict__ Xp, int64_t rows,
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
    // piece's address is this lane's offset plus a wave-uniform one plus the
    // step's k-block.
    const int g = (lane & 3) ^ ((lane >> 4) & 3);
    const __bf16 *lane_src = Xp + (lane >> 2) * XB_K + 8 * g;
    auto wave_off = [&](int v) __attribute__((always_inline)) -> int64_t {
        const int b = 4 * v + w, rb = b & 15;
        const int row0 = (rb < 8) ? m0 + 16 * rb : n0 + 16 * (rb - 8);
        return (int64_t)(b >> 4) * plane + row0 * XB_K;
    };
    // a full step straight into LDS (12 loads per lane); a partial last step
    // through registers with the values past ke set to zero
    auto load_step = [&](__bf16 *stage, int64_t k0) __attribute__((always_inline)) {
        const int64_t kblk = (k0 / XB_K) * (rows * XB_K);
        if (k0 + BX_TK <= ke) {
#pragma unroll
            for (int v = 0; v < BX_LOADS; ++v)
                lds_dma16(lane_src + wave_off(v) + kblk, (lds_void *)(stage + 512 * (4 * v + w)));
        } else {
#pragma unroll
            for (int v = 0; v < BX_LOADS; ++v) {
                const __bf16 *src = lane_src + wave_off(v) + kblk;
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

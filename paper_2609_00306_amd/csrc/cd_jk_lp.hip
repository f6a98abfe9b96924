// Reduced-precision forms of the exchange build (K), with FP32 accumulation
// inside k-slabs of 32 and FP64 accumulation across slabs; J is always built
// in FP64 (it is bound by reading L).
//
//   FP32  : the half transform X^P = Lt^P C and the product K = sum_P X^P^T X^P
//           both on v_mfma_f32_16x16x4f32, operands rounded to FP32 on load.
//   BF16X3: the half transform runs in FP64 and writes X split into three BF16
//           planes (k_half_sparse<true>); the product K reads the planes
//           (k_syrk_rows_bf16p).  Every operand x is split as x = b0 + b1 + b2 (round-to-nearest
//           BF16 each: b0 = bf16(x), b1 = bf16(x - b0), b2 = bf16(x - b0 - b1)),
//           and a product a*c keeps the six terms up to order 2^-16:
//           a0c0 + a0c1 + a1c0 + a0c2 + a1c1 + a2c0  (Henry, Tang & Heinecke,
//           "Leveraging the bfloat16 artificial intelligence datatype for
//           higher-precision computations", ARITH 2019), on
//           v_mfma_f32_16x16x32_bf16.
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

enum LpMode { LP_F32 = 1, LP_BF16X3 = 2 };

constexpr int LP_TKC = 32;     // k-chunk staged in LDS
constexpr int LP_SLAB = 32;    // FP32 accumulation length before folding into FP64

__device__ __forceinline__ int lp_row(int lane, int v) { return 4 * (lane >> 4) + v; }

__device__ __forceinline__ void split3(double x, __bf16 &b0, __bf16 &b1, __bf16 &b2)
{
    b0 = (__bf16)(float)x;
    const double r1 = x - (double)(float)b0;
    b1 = (__bf16)(float)r1;
    const double r2 = r1 - (double)(float)b1;
    b2 = (__bf16)(float)r2;
}

// LDS staging of one k-chunk for a 64 x 64 tile.
//  F32 : k-major sources   sA32[k][m], sB32[k][n]
//        k-contiguous (KC) sA32[m][k], sB32[n][k]  (rows padded to TKC + 1)
//  BF16: sAp[p][m][k], sBp[p][n][k] p = 0..2    (k contiguous, 8 per lane load)
// so that the LDS writes follow the contiguous index of the global loads.
template <int MODE, bool KC = false>
struct LpStage {
    static constexpr int kBf16Ld = LP_TKC + 8;   // padded row (bf16 elements)
    static constexpr int kF32Ld = LP_TKC + 1;    // padded row (KC, FP32)
    static constexpr int kBytes = (MODE == LP_F32) ? 2 * 64 * (LP_TKC + 1) * 4
                                                   : 2 * 3 * 64 * kBf16Ld * 2;
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
        if (MODE == LP_F32) {
            float *sA = reinterpret_cast<float *>(smem);
            float *sB = sA + 64 * kF32Ld;
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                int k, m;
                coord(threadIdx.x + 256 * u, k, m);
                sA[f32_index(k, m)] = (float)ra[u];
                sB[f32_index(k, m)] = (float)rb[u];
            }
        } else {
            __bf16 *sA = reinterpret_cast<__bf16 *>(smem);
            __bf16 *sB = sA + 3 * 64 * kBf16Ld;
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                int k, m;
                coord(threadIdx.x + 256 * u, k, m);
                __bf16 a0, a1, a2, c0, c1, c2;
                split3(ra[u], a0, a1, a2);
                split3(rb[u], c0, c1, c2);
                sA[(0 * 64 + m) * kBf16Ld + k] = a0;
                sA[(1 * 64 + m) * kBf16Ld + k] = a1;
                sA[(2 * 64 + m) * kBf16Ld + k] = a2;
                sB[(0 * 64 + m) * kBf16Ld + k] = c0;
                sB[(1 * 64 + m) * kBf16Ld + k] = c1;
                sB[(2 * 64 + m) * kBf16Ld + k] = c2;
            }
        }
    }
    // multiply the staged chunk into acc[r] (rows 16 r.., columns 16 w..)
    __device__ static __forceinline__ void mma(const unsigned char *smem, f32x4 (&acc)[4])
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        if (MODE == LP_F32) {
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
        } else {
            mma_planes(reinterpret_cast<const __bf16 *>(smem),
                       reinterpret_cast<const __bf16 *>(smem) + 3 * 64 * kBf16Ld, acc);
        }
    }
    // BF16 planes sA[p][m][k], sB[p][n][k] (k contiguous, rows of kBf16Ld): the
    // six products of the 3 x BF16 split into acc[r] (rows 16 r.., columns 16 w..)
    __device__ static __forceinline__ void mma_planes(const __bf16 *sA, const __bf16 *sB,
                                                      f32x4 (&acc)[4])
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        {
            const int kk = 8 * (lane >> 4);
            bf16x8 b[3];
#pragma unroll
            for (int p = 0; p < 3; ++p)
                b[p] = *reinterpret_cast<const bf16x8 *>(
                    &sB[(p * 64 + 16 * w + (lane & 15)) * kBf16Ld + kk]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                bf16x8 a[3];
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    a[p] = *reinterpret_cast<const bf16x8 *>(
                        &sA[(p * 64 + 16 * r + (lane & 15)) * kBf16Ld + kk]);
                // smallest terms first
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], acc[r], 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], acc[r], 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], acc[r], 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], acc[r], 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], acc[r], 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], acc[r], 0, 0, 0);
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

// Half transform over neighbour lists, reduced precision, FP32 out:
//   Y[mu][P * ncol + i] = sum_{j in nbr(mu)} LT[r_j][P] C[sigma_j][i]
template <int MODE>
__global__ __launch_bounds__(256) void k_half_sparse_lp(const double *__restrict__ LT, int64_t ldt,
                                                        const int64_t *__restrict__ off,
                                                        const int32_t *__restrict__ nb_s,
                                                        const int32_t *__restrict__ nb_r,
                                                        const double *__restrict__ C, int ncol,
                                                        const int64_t *__restrict__ n_vectors,
                                                        float *__restrict__ Y, int64_t ldy)
{
    __shared__ __align__(16) unsigned char smem[LpStage<MODE>::kBytes];
    const int64_t M = *n_vectors;
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    if (p0 >= M) return;
    const int n0 = blockIdx.y * 64;
    const int mu = blockIdx.z;
    const int64_t j0 = off[mu], deg = off[mu + 1] - j0;
    double acc[4][4] = {};
    __shared__ int sNs[NB_SEG], sNr[NB_SEG];   // neighbour list, staged in segments
    for (int64_t seg = 0; seg < deg; seg += NB_SEG) {
        const int len = (int)min((int64_t)NB_SEG, deg - seg);
        __syncthreads();
        for (int e = threadIdx.x; e < len; e += 256) {
            sNs[e] = nb_s[j0 + seg + e];
            sNr[e] = nb_r[j0 + seg + e];
        }
        __syncthreads();
        lp_tile<MODE, false>(
            seg, seg + len,
            [&](int64_t k, int m) -> double {
                return LT[(int64_t)sNr[k - seg] * ldt + min(p0 + m, M - 1)];
            },
            [&](int64_t k, int n) -> double {
                return C[(int64_t)sNs[k - seg] * ncol + min(n0 + n, ncol - 1)];
            },
            acc, smem);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float *out = Y + (int64_t)mu * ldy;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t P = p0 + 16 * r + lp_row(lane, v);
            const int i = n0 + 16 * w + (lane & 15);
            if (P < M && i < ncol) out[P * ncol + i] = (float)acc[r][v];
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

// Partial K from X held as three BF16 planes (written by the FP64 half
// transform): Kp[s][mu][nu] = sum_{k in slab s} X[mu][k] X[nu][k] with the six
// products of the 3 x BF16 split, FP32 inside each 32-k chunk, FP64 across.
// Each thread loads one 16-byte piece (8 values) of one row per plane and
// operand; ldx is a multiple of 8 so the pieces are aligned.
__global__ __launch_bounds__(256) void k_syrk_rows_bf16p(const __bf16 *__restrict__ Xp,
                                                         int64_t ldx, int64_t plane, int N,
                                                         const int64_t *__restrict__ n_vectors,
                                                         int ncol, int nsplit,
                                                         double *__restrict__ Kp)
{
    using S = LpStage<LP_BF16X3, true>;
    constexpr int LD = S::kBf16Ld;
    __shared__ __align__(16) __bf16 sA[3 * 64 * LD];
    __shared__ __align__(16) __bf16 sB[3 * 64 * LD];
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
    const int tid = threadIdx.x, row = tid >> 2, kv = 8 * (tid & 3);
    const __bf16 *pa = Xp + (int64_t)min(m0 + row, N - 1) * ldx + kv;
    const __bf16 *pb = Xp + (int64_t)min(n0 + row, N - 1) * ldx + kv;
    double acc64[4][4] = {};
    f32x4 acc[4];
    bf16x8 va[3], vb[3];
    auto fetch = [&](int64_t k0) {
        if (k0 + kv + 8 <= ke) {
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                va[p] = *reinterpret_cast<const bf16x8 *>(pa + p * plane + k0);
                vb[p] = *reinterpret_cast<const bf16x8 *>(pb + p * plane + k0);
            }
        } else {
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bool ok = k0 + kv + j < ke;
                    va[p][j] = ok ? pa[p * plane + k0 + j] : (__bf16)0.0f;
                    vb[p][j] = ok ? pb[p * plane + k0 + j] : (__bf16)0.0f;
                }
        }
    };
    if (kb < ke) fetch(kb);
    for (int64_t k0 = kb; k0 < ke; k0 += LP_TKC) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            *reinterpret_cast<bf16x8 *>(&sA[(p * 64 + row) * LD + kv]) = va[p];
            *reinterpret_cast<bf16x8 *>(&sB[(p * 64 + row) * LD + kv]) = vb[p];
        }
        __syncthreads();
        if (k0 + LP_TKC < ke) fetch(k0 + LP_TKC);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = f32x4{0.f, 0.f, 0.f, 0.f};
        S::mma_planes(sA, sB, acc);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[r][v] += (double)acc[r][v];
    }
    const int lane = tid & 63, w = tid >> 6;
    double *out = Kp + (int64_t)s * N * N;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = m0 + 16 * r + lp_row(lane, v), n = n0 + 16 * w + (lane & 15);
            if (m < N && n < N) out[(int64_t)m * N + n] = acc64[r][v];
        }
}

}  // namespace cdk

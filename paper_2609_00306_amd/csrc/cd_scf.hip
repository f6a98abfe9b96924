// Closed-shell SCF on Cholesky J/K (Sec. 4.1): the one-electron integrals
// over the s functions, and the dense N x N building blocks of a
// diagonalisation-free Roothaan-Hall step.
//
//   one-electron : S, T and the attraction to point charges in closed form
//                  (textbook s-function formulas with the Boys function F0);
//   orthogonaliser: X = S^{-1/2} by the coupled Newton-Schulz iteration
//                  Y <- Y T, Z <- T Z, T = (3 I - Z Y) / 2 from Y = S / c,
//                  Z = I (c bounds the spectrum of S from above);
//   density      : the projector on the O lowest solutions of F C = S C e,
//                  by trace-correcting purification of X F X (Niklasson,
//                  Phys. Rev. B 66, 155115 (2002)): P <- P^2 when tr P > O,
//                  else 2 P - P^2 (the branch taken on the device), from
//                  P0 = (l_max - X F X) / (l_max - l_min) with Gershgorin
//                  bounds; D = X P X;
//   orbitals     : D = C C^T with C [N][O] from a pivoted Cholesky
//                  decomposition of the rank-O density (any such C gives the
//                  same J and K, which depend on D only);
//   extrapolation: Pulay's DIIS over the last 8 Fock matrices with the
//                  commutators F D S - S D F as error vectors (the small
//                  bordered system is solved on the host).
// Every product is an FP64 matrix-core GEMM (the shared tile engine); every
// sum over matrix elements runs in a fixed order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "cd_device.hpp"
#include "cd_mfma.hpp"

namespace cdk {

// ---------------------------------------------------------------- one-electron
// S_ab = N_a N_b (pi/p)^{3/2} exp(-m R^2), T_ab = m (3 - 2 m R^2) S_ab,
// V_ab = -sum_C Z_C 2 pi / p N_a N_b exp(-m R^2) F0(p |P - C|^2),
// p = a + b, m = a b / p, P = (a A + b B) / p, N = (2 x / pi)^{3/4}.
__global__ __launch_bounds__(256) void k_one_electron(int N, const double *__restrict__ xyz,
                                                      const double *__restrict__ alpha, int nc,
                                                      const double *__restrict__ cxyz,
                                                      const double *__restrict__ Z,
                                                      double *__restrict__ S,
                                                      double *__restrict__ H)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    const int a = (int)(e / N), b = (int)(e % N);
    const double xa = alpha[a], xb = alpha[b];
    const double p = xa + xb, m = xa * xb / p;
    double r2 = 0.0, P[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double A = xyz[3 * a + k], B = xyz[3 * b + k];
        r2 += (A - B) * (A - B);
        P[k] = (xa * A + xb * B) / p;
    }
    const double nn = pow(2.0 * xa / kPi, 0.75) * pow(2.0 * xb / kPi, 0.75);
    const double E = nn * exp(-m * r2);
    const double s = E * pow(kPi / p, 1.5);
    double v = 0.0;
    for (int c = 0; c < nc; ++c) {
        double pc2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double d = P[k] - cxyz[3 * c + k];
            pc2 += d * d;
        }
        v -= Z[c] * (2.0 * kPi / p) * E * boys0(p * pc2);
    }
    S[e] = s;
    H[e] = m * (3.0 - 2.0 * m * r2) * s + v;
}

// ---------------------------------------------------------------- dense GEMM
// C = A B for row-major N x N matrices: one 64 x 64 tile per workgroup; with
// gridDim.z > 1 workgroup z takes the k-range [z kchunk, (z + 1) kchunk) and
// writes its partial product to C + z N^2 (added by k_sum_split), so a small
// N still fills the compute units.
constexpr int SCF_TKC = 32;
constexpr int SCF_KSPLIT_MAX = 8;
__global__ __launch_bounds__(256) void k_gemm_nn(int N, const double *__restrict__ A,
                                                 const double *__restrict__ B,
                                                 double *__restrict__ C, int kchunk)
{
    using SA = OperandStage<64, SCF_TKC, false>;
    using SB = OperandStage<64, SCF_TKC, true>;
    __shared__ double sA[SA::kSize];
    __shared__ double sB[SB::kSize];
    const int r0 = 64 * blockIdx.y, c0 = 64 * blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kb = blockIdx.z * kchunk, ke = min(N, kb + kchunk);
    C += (int64_t)blockIdx.z * N * N;
    f64x4 acc[4];
    zero_acc(acc);
    gemm_tile<4, SCF_TKC, false, true>(
        kb, ke,
        [&](int64_t k, int m) -> double {
            const int r = r0 + m;
            return (r < N) ? A[(int64_t)r * N + k] : 0.0;
        },
        [&](int64_t k, int n) -> double {
            const int c = c0 + n;
            return (c < N) ? B[k * N + c] : 0.0;
        },
        acc, sA, sB);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = r0 + 16 * r + mfma_row(lane, v), col = c0 + 16 * w + (lane & 15);
            if (row < N && col < N) C[(int64_t)row * N + col] = acc[r][v];
        }
}

// C[e] = sum_z part[z n2 + e], z ascending
__global__ __launch_bounds__(256) void k_sum_split(int64_t n2, int ks, const double *__restrict__ part,
                                                   double *__restrict__ C)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n2) return;
    double v = part[e];
    for (int z = 1; z < ks; ++z) v += part[(int64_t)z * n2 + e];
    C[e] = v;
}

// out = a X + b Y + c I (Y may be null when b == 0)
// (out may be X or Y: each element is read before it is written by the same thread)
__global__ __launch_bounds__(256) void k_lincomb(int N, double *out, double a, const double *X,
                                                 double b, const double *Y, double c)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    double v = a * X[e];
    if (Y) v += b * Y[e];
    if (e / N == e % N) v += c;
    out[e] = v;
}

// One trace-correcting purification step, the branch taken from tr P
// (tr[0], written by k_traces): P <- P^2 when tr P > O, else 2 P - P^2.
__global__ __launch_bounds__(256) void k_tc2_step(int N, double *P, const double *P2,
                                                  const double *tr, double occ)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    const double q = P2[e];
    P[e] = (tr[0] > occ) ? q : 2.0 * P[e] - q;
}

// Fixed-order sum and max of one value per thread of a 256-thread workgroup
// (valid in thread 0).
__device__ __forceinline__ double scf_block_sum(double v, double *s)
{
    const int tid = threadIdx.x;
    __syncthreads();
    s[tid] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) s[tid] = s[tid] + s[tid + w];
        __syncthreads();
    }
    return s[0];
}

__device__ __forceinline__ double scf_block_max(double v, double *s)
{
    const int tid = threadIdx.x;
    __syncthreads();
    s[tid] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) s[tid] = fmax(s[tid], s[tid + w]);
        __syncthreads();
    }
    return s[0];
}

// out[0] = tr X, out[1] = tr Y (one workgroup)
__global__ __launch_bounds__(256) void k_traces(int N, const double *__restrict__ X,
                                                const double *__restrict__ Y,
                                                double *__restrict__ out)
{
    __shared__ double s[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < N; i += 256) {
        a += X[(int64_t)i * N + i];
        b += Y[(int64_t)i * N + i];
    }
    const double ta = scf_block_sum(a, s);
    const double tb = scf_block_sum(b, s);
    if (threadIdx.x == 0) {
        out[0] = ta;
        out[1] = tb;
    }
}

// *out = max |G - G^T| (the commutator F D S - S D F with G = F D S for
// symmetric F, D, S), or with 'minus_identity' max |G - I|.  Grid-stride over
// the N^2 elements; the maximum of non-negative doubles is taken on their bit
// patterns (which order like the values), so the result does not depend on
// the order.  *out must hold +0.0 before the launch.
__global__ __launch_bounds__(256) void k_maxabs(int N, const double *__restrict__ G,
                                                int minus_identity, double *__restrict__ out)
{
    const int64_t n2 = (int64_t)N * N;
    double m = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / N), j = (int)(e % N);
        const double v = minus_identity ? G[e] - (i == j ? 1.0 : 0.0)
                                        : G[e] - G[(int64_t)j * N + i];
        m = (v != v) ? INFINITY : fmax(m, fabs(v));   // a NaN reads as unbounded
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(out),
                  (unsigned long long)__double_as_longlong(m));
}

// Fixed-order sums of 'nb' partials per row: out[b] = sum_k part[b * nb + k]
// (one workgroup per row b), plus 'add'.
__global__ __launch_bounds__(256) void k_sum_partials(int nb, const double *__restrict__ part,
                                                      double add, double *__restrict__ out)
{
    __shared__ double s[256];
    double a = 0.0;
    for (int k = threadIdx.x; k < nb; k += 256) a += part[(int64_t)blockIdx.x * nb + k];
    const double t = scf_block_sum(a, s);
    if (threadIdx.x == 0) out[blockIdx.x] = t + add;
}

// Gershgorin bounds of a symmetric matrix, one wave per row: keys[0] and
// keys[1] collect, on order-preserving integer keys, the smallest d - r and
// the largest d + r (d the diagonal element, r the off-diagonal absolute row
// sum).  keys[0] must start at all ones and keys[1] at zero.
__device__ __forceinline__ unsigned long long order_key(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__host__ __device__ inline double key_value(unsigned long long k)
{
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double x;
    memcpy(&x, &b, sizeof x);
    return x;
}

__global__ __launch_bounds__(256) void k_gershgorin(int N, const double *__restrict__ A,
                                                    unsigned long long *__restrict__ keys)
{
    const int lane = threadIdx.x & 63;
    const int row = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (row >= N) return;
    double r = 0.0;
    for (int j = lane; j < N; j += 64)
        if (j != row) r += fabs(A[(int64_t)row * N + j]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) r += __shfl_xor(r, off, 64);
    if (lane == 0) {
        const double d = A[(int64_t)row * N + row];
        atomicMin(&keys[0], order_key(d - r));
        atomicMax(&keys[1], order_key(d + r));
    }
}

__global__ void k_gershgorin_init(unsigned long long *keys)
{
    keys[0] = ~0ull;
    keys[1] = 0ull;
}

// F = H + 2 J - K, and per workgroup the fixed-order partial sum of
// D o (H + F) (grid-stride over the N^2 elements with a fixed grid, so the
// partition, and with k_sum_partials the energy, is the same on every run).
__global__ __launch_bounds__(256) void k_fock_energy(int N, const double *__restrict__ H,
                                                     const double *__restrict__ J,
                                                     const double *__restrict__ K,
                                                     const double *__restrict__ D,
                                                     double *__restrict__ F,
                                                     double *__restrict__ part)
{
    __shared__ double s[256];
    double acc = 0.0;
    const int64_t n2 = (int64_t)N * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double f = H[e] + 2.0 * J[e] - K[e];
        F[e] = f;
        acc += D[e] * (H[e] + f);
    }
    const double t = scf_block_sum(acc, s);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Pulay extrapolation (DIIS) of the Fock matrix over stored iterations.
constexpr int SCF_DIIS = 8;
struct DiisCoef {
    double c[SCF_DIIS];
    int slot[SCF_DIIS];
    int n;
};

// e = G - G^T (the commutator F D S - S D F for G = F D S); also copies F into
// the history slot
__global__ __launch_bounds__(256) void k_diis_store(int N, const double *__restrict__ G,
                                                    const double *__restrict__ F,
                                                    double *__restrict__ e_out,
                                                    double *__restrict__ f_out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    const int i = (int)(e / N), j = (int)(e % N);
    e_out[e] = G[e] - G[(int64_t)j * N + i];
    f_out[e] = F[e];
}

// part[b * gridDim.x + x] = the fixed-order partial sum, over workgroup x's
// share of the N^2 elements, of e_new o hist[slot[b]] (grid: x, b); the
// overlaps follow from k_sum_partials
__global__ __launch_bounds__(256) void k_diis_dots(int64_t n2, const double *__restrict__ e_new,
                                                   const double *__restrict__ hist,
                                                   const DiisCoef slots,
                                                   double *__restrict__ part)
{
    __shared__ double s[256];
    const int b = blockIdx.y;
    if (b >= slots.n) return;
    const double *h = hist + (int64_t)slots.slot[b] * n2;
    double a = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
         e += (int64_t)gridDim.x * blockDim.x)
        a += e_new[e] * h[e];
    const double t = scf_block_sum(a, s);
    if (threadIdx.x == 0) part[(int64_t)b * gridDim.x + blockIdx.x] = t;
}

// F = sum_b c[b] hist[slot[b]]
__global__ __launch_bounds__(256) void k_diis_combine(int64_t n2, const double *__restrict__ hist,
                                                      const DiisCoef co, double *__restrict__ F)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n2) return;
    double v = 0.0;
    for (int b = 0; b < co.n; ++b) v += co.c[b] * hist[(int64_t)co.slot[b] * n2 + e];
    F[e] = v;
}

// C [N][O] with C C^T = D for the rank-O density D: a pivoted Cholesky
// decomposition taking the O largest residual diagonals in turn (lowest index
// on ties).  One 1024-thread workgroup; the columns are formed in 'Ct' [O][N]
// (so each is written and read with consecutive rows on consecutive threads)
// and copied to C at the end; 'dres' [N] is scratch.  Status 4 when a pivot is
// not positive.
constexpr int DCH_T = 1024;
__global__ __launch_bounds__(DCH_T) void k_density_cholesky(int N, int O,
                                                            const double *__restrict__ D,
                                                            double *__restrict__ Ct,
                                                            double *__restrict__ C,
                                                            double *__restrict__ dres,
                                                            int32_t *__restrict__ status)
{
    __shared__ double sv[DCH_T];
    __shared__ int si[DCH_T];
    __shared__ double sp[1024];   // Ct[j][p] for the current pivot, j < k (chunks of 1024)
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += DCH_T) dres[i] = D[(int64_t)i * N + i];
    __syncthreads();
    int kdone = O;
    for (int k = 0; k < O; ++k) {
        double bv = -INFINITY;
        int bi = N;
        for (int i = tid; i < N; i += DCH_T) {
            const double d = dres[i];
            if (d > bv) {   // ascending i per thread: the first maximum stays
                bv = d;
                bi = i;
            }
        }
        sv[tid] = bv;
        si[tid] = bi;
        __syncthreads();
        for (int w = DCH_T / 2; w > 0; w >>= 1) {
            if (tid < w) {
                const double ov = sv[tid + w];
                const int oi = si[tid + w];
                if (ov > sv[tid] || (ov == sv[tid] && oi < si[tid])) {
                    sv[tid] = ov;
                    si[tid] = oi;
                }
            }
            __syncthreads();
        }
        const int p = si[0];
        const double dp = sv[0];
        if (!(dp > 0.0) || p >= N) {
            if (tid == 0) status[0] = 4;
            kdone = k;
            break;
        }
        const double inv = 1.0 / sqrt(dp);
        double v[4];
        for (int i0 = 0; i0 < N; i0 += 4 * DCH_T) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + tid + u * DCH_T;
                v[u] = (i < N) ? D[(int64_t)i * N + p] : 0.0;
            }
            for (int j0 = 0; j0 < k; j0 += 1024) {
                const int nj = min(1024, k - j0);
                __syncthreads();
                if (tid < nj) sp[tid] = Ct[(int64_t)(j0 + tid) * N + p];
                __syncthreads();
                for (int j = 0; j < nj; ++j) {
                    const double c = sp[j];
                    const double *row = Ct + (int64_t)(j0 + j) * N;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = i0 + tid + u * DCH_T;
                        if (i < N) v[u] = fma(-row[i], c, v[u]);
                    }
                }
            }
            __syncthreads();   // every read of column p's earlier entries is done
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + tid + u * DCH_T;
                if (i < N) {
                    const double l = v[u] * inv;
                    Ct[(int64_t)k * N + i] = l;
                    dres[i] = (i == p) ? -INFINITY : dres[i] - l * l;
                }
            }
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)N * O; e += DCH_T) {
        const int i = (int)(e / O), j = (int)(e % O);
        C[e] = (j < kdone) ? Ct[(int64_t)j * N + i] : 0.0;
    }
}

}  // namespace cdk

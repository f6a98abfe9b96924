// Coulomb/exchange builds from the Cholesky vectors (paper Sec. 4.1: J costs
// O(N^2 M), K costs O(O N^2 M)) and the AO->MO transform of the vectors
// (Sec. 4.1, CASSCF; two-coefficient form of Sec. 9).
//
//   J_{mu nu} = sum_P L^P_{mu nu} V^P,  V^P = sum_{rho sigma} L^P_{rho sigma} D_{rho sigma},  D = C C^T
//   K_{mu nu} = sum_P sum_i X^P_{i mu} X^P_{i nu},  X^P_{i mu} = sum_sigma L^P_{mu sigma} C_{sigma i}
//   Lmo^P_{ab} = sum_{mu nu} C1_{mu a} L^P_{mu nu} C2_{nu b}
//
// L is packed over screened pairs (rows); a dense N x N row map unpacks it
// on the fly into the MFMA operand tiles.
#include "cd_device.hpp"
#include "cd_mfma.hpp"

namespace cdk {

__global__ void k_fill_f64(double *__restrict__ p, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// rowof[mu][nu] = rowof[nu][mu] = row of pair (mu, nu), -1 if screened out
__global__ void k_rowmap(int64_t n_rows, const int64_t *__restrict__ row_pair, int N,
                         int32_t *__restrict__ rowof)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    int mu, nu;
    unpack_pair(row_pair[r], mu, nu);
    rowof[(int64_t)mu * N + nu] = (int32_t)r;
    rowof[(int64_t)nu * N + mu] = (int32_t)r;
}

// D = C C^T  ([N][N], C [N][O])
__global__ void k_density(int N, int O, const double *__restrict__ C, double *__restrict__ Dm)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    int a = (int)(e / N), b = (int)(e % N);
    double s = 0.0;
    for (int i = 0; i < O; ++i) s = fma(C[(int64_t)a * O + i], C[(int64_t)b * O + i], s);
    Dm[e] = s;
}

// w[r] = (2 - delta_{mu nu}) D_{mu nu}: the packed-row weight of the density
__global__ void k_drow(int64_t n_rows, const int64_t *__restrict__ row_pair, int N,
                       const double *__restrict__ Dm, double *__restrict__ w)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    int mu, nu;
    unpack_pair(row_pair[r], mu, nu);
    double d = Dm[(int64_t)mu * N + nu];
    w[r] = (mu == nu) ? d : 2.0 * d;
}

// V[P] = sum_r L[P][r] w[r]  (one workgroup per vector)
__global__ __launch_bounds__(256) void k_jV(const double *__restrict__ L, int64_t n_rows,
                                            const double *__restrict__ w,
                                            const int64_t *__restrict__ n_vectors,
                                            double *__restrict__ V)
{
    __shared__ double s_part[4];
    const int64_t Pv = blockIdx.x;
    if (Pv >= *n_vectors) return;
    const double *row = L + Pv * n_rows;
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n_rows; r += 256) s = fma(row[r], w[r], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) V[Pv] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

// J at row r = sum_P L[P][r] V[P]; written to both (mu,nu) and (nu,mu)
__global__ __launch_bounds__(256) void k_jJ(const double *__restrict__ L, int64_t n_rows,
                                            const double *__restrict__ V,
                                            const int64_t *__restrict__ n_vectors,
                                            const int64_t *__restrict__ row_pair, int N,
                                            double *__restrict__ J)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int64_t M = *n_vectors;
    double s = 0.0;
    for (int64_t Pv = 0; Pv < M; ++Pv) s = fma(L[Pv * n_rows + r], V[Pv], s);
    int mu, nu;
    unpack_pair(row_pair[r], mu, nu);
    J[(int64_t)mu * N + nu] = s;
    J[(int64_t)nu * N + mu] = s;
}

// Half transform Y^P = Lt^P C  (Lt^P the unpacked symmetric N x N vector):
//   Y^P[mu][i] = sum_sigma Lt^P[sigma][mu] C[sigma][i]
// tile: m = mu, n = i, k = sigma.  Output layout:
//   TRANSPOSED: Y[(P * ncol + i) * N + mu]   (k-major rows for the K product)
//   else      : Y[(P * N + mu) * ncol + i]
template <bool TRANSPOSED>
__global__ __launch_bounds__(256) void k_half(const double *__restrict__ L, int64_t n_rows,
                                              const int32_t *__restrict__ rowof, int N,
                                              const double *__restrict__ C, int ncol,
                                              const int64_t *__restrict__ n_vectors,
                                              int64_t p_base, double *__restrict__ Y)
{
    __shared__ double sA[TK * TM];
    __shared__ double sB[TK * TN];
    __shared__ double sT[TM][TN + 1];
    const int64_t Pv = p_base + blockIdx.z;
    if (Pv >= *n_vectors) return;
    const int m0 = blockIdx.x * TM;
    const int n0 = blockIdx.y * TN;
    const double *Lp = L + Pv * n_rows;
    TileAcc acc;
    acc.zero();
    mfma_tile_f64(
        0, N,
        [&](int64_t k, int m) -> double {
            int mu = m0 + m;
            if (mu >= N) return 0.0;
            int32_t r = rowof[k * N + mu];
            return (r >= 0) ? Lp[r] : 0.0;
        },
        [&](int64_t k, int n) -> double {
            int i = n0 + n;
            return (i < ncol) ? C[k * ncol + i] : 0.0;
        },
        acc, sA, sB);
    tile_to_lds(acc, &sT[0][0], TN + 1);
    __syncthreads();
    const int64_t Yb = (Pv - p_base);
    for (int e = threadIdx.x; e < TM * TN; e += 256) {
        if (TRANSPOSED) {
            int n = e / TM, m = e % TM;
            if (m0 + m < N && n0 + n < ncol)
                Y[(Yb * ncol + n0 + n) * (int64_t)N + m0 + m] = sT[m][n];
        } else {
            int m = e / TN, n = e % TN;
            if (m0 + m < N && n0 + n < ncol)
                Y[(Yb * N + m0 + m) * (int64_t)ncol + n0 + n] = sT[m][n];
        }
    }
}

// Partial K over a k-slab: Kp[s][mu][nu] = sum_{k in slab s} X[k][mu] X[k][nu]
// for lower tile pairs (tm >= tn); X is [nk][N].
__global__ __launch_bounds__(256) void k_syrk(const double *__restrict__ X, int N,
                                              const int64_t *__restrict__ n_vectors, int ncol,
                                              int64_t p_base, int64_t p_count, int nsplit,
                                              double *__restrict__ Kp)
{
    __shared__ double sA[TK * TM];
    __shared__ double sB[TK * TN];
    // tile pair from blockIdx.x: tm >= tn
    int t = blockIdx.x;
    int tm = 0;
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    int tn = t - tm * (tm + 1) / 2;
    const int s = blockIdx.y;
    int64_t M = *n_vectors - p_base;
    if (M > p_count) M = p_count;
    if (M < 0) M = 0;
    const int64_t nk = M * ncol;
    int64_t per = (nk + nsplit - 1) / nsplit;
    per = (per + TK - 1) / TK * TK;
    const int64_t kb = s * per;
    const int64_t ke = (kb + per < nk) ? kb + per : nk;
    TileAcc acc;
    acc.zero();
    const int m0 = tm * TM, n0 = tn * TN;
    if (kb < ke)
        mfma_tile_f64(
            kb, ke,
            [&](int64_t k, int m) -> double {
                return (m0 + m < N) ? X[k * N + m0 + m] : 0.0;
            },
            [&](int64_t k, int n) -> double {
                return (n0 + n < N) ? X[k * N + n0 + n] : 0.0;
            },
            acc, sA, sB);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    double *out = Kp + (int64_t)s * N * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int m = m0 + wm + 16 * i + mfma_row(lane, v);
                int n = n0 + wn + 16 * j + (lane & 15);
                if (m < N && n < N) out[(int64_t)m * N + n] = acc.c[i][j][v];
            }
}

// K[mu][nu] (+)= sum_s Kp[s][max][min]  -- exactly symmetric
__global__ void k_kreduce(const double *__restrict__ Kp, int N, int nsplit, int accumulate,
                          double *__restrict__ K)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    int mu = (int)(e / N), nu = (int)(e % N);
    int a = mu > nu ? mu : nu, b = mu > nu ? nu : mu;
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s += Kp[(int64_t)sp * N * N + (int64_t)a * N + b];
    K[e] = accumulate ? K[e] + s : s;
}

// Lmo[P][a][b] = sum_mu C1[mu][a] Y[P][mu][b]   (Y from k_half<false> with C2)
__global__ __launch_bounds__(256) void k_tr2(const double *__restrict__ Y, int N,
                                             const double *__restrict__ C1, int p, int q,
                                             const int64_t *__restrict__ n_vectors,
                                             int64_t p_base, double *__restrict__ Lmo)
{
    __shared__ double sA[TK * TM];
    __shared__ double sB[TK * TN];
    const int64_t Pv = p_base + blockIdx.z;
    if (Pv >= *n_vectors) return;
    const int m0 = blockIdx.x * TM;   // a
    const int n0 = blockIdx.y * TN;   // b
    const double *Yp = Y + (Pv - p_base) * (int64_t)N * q;
    TileAcc acc;
    acc.zero();
    mfma_tile_f64(
        0, N,
        [&](int64_t k, int m) -> double { return (m0 + m < p) ? C1[k * p + m0 + m] : 0.0; },
        [&](int64_t k, int n) -> double { return (n0 + n < q) ? Yp[k * q + n0 + n] : 0.0; },
        acc, sA, sB);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    double *out = Lmo + Pv * (int64_t)p * q;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int a = m0 + wm + 16 * i + mfma_row(lane, v);
                int b = n0 + wn + 16 * j + (lane & 15);
                if (a < p && b < q) out[(int64_t)a * q + b] = acc.c[i][j][v];
            }
}

}  // namespace cdk

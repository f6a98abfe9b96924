// Pivoted Cholesky decomposition of a complex Hermitian positive semidefinite
// matrix (the finite-field case of Sec. 7: the integrals over field-dependent
// orbitals are complex, the matrix is Hermitian with a real diagonal, and the
// vectors are complex with A ~ sum_K L_K L_K^H).  Sec. 2 in complex algebra:
//     P_K = argmax_r D_r (lowest r on ties),  d_K = D_{P_K},
//     L^K_r = [ A_{r P_K} - sum_{J<K} L^J_r conj(L^J_{P_K}) ] / sqrt(d_K),
//     D_r -= |L^K_r|^2,  D_{P_K} = 0,  stop when d_K < tau.
//
// One persistent cooperative kernel runs the whole loop with one grid barrier
// per vector.  Workgroup g owns R consecutive rows (R a power of two, at most
// 256); its 256 threads are R rows x (256 / R) k-lanes, rows fastest, so for
// every earlier vector J the R rows of a workgroup read R contiguous complex
// values.  The k-lanes' partial sums are added in LDS in a fixed order.  The
// column A(:, P_K) is read as the conjugate of row P_K (contiguous).  Every
// workgroup leaves the largest updated residual of its rows (and its row) in
// a double-buffered slot; after the barrier every workgroup reduces the slots
// the same way and so agrees on the next pivot and on when to stop.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cd_device.hpp"

namespace cdk {

struct ZcdParams {
    int64_t n;
    const double2 *A;          // [n][n] Hermitian (row-major)
    double tau;
    int64_t max_vectors;
    double2 *L;                // [max_vectors][n]
    int64_t *pivots;           // [max_vectors]
    double *D;                 // [n] residual diagonal
    int64_t *n_vectors;        // [1]
    int32_t *status;           // [1]
    GridSync *gs;
    Nom *part;                 // [2][G] per-workgroup largest residual
    int32_t G;                 // workgroups taking part
    int32_t R;                 // rows per workgroup (power of two, <= 256)
    uint32_t spin_limit;
};

__device__ __forceinline__ void zcd_better(double &bd, int &bi, double d, int i)
{
    if (nom_before(d, i, bd, bi)) {
        bd = d;
        bi = i;
    }
}

// Butterfly max of (d, idx) over the 64 lanes of a wave, lowest idx on ties
// (a total order, so every lane ends with the same pair).
__device__ __forceinline__ void zcd_wave_max(double &d, int &i)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double od = __shfl_xor(d, off, 64);
        const int oi = __shfl_xor(i, off, 64);
        zcd_better(d, i, od, oi);
    }
}

// Largest of one (d, idx) per thread over the 256-thread workgroup: a wave
// butterfly, then the four wave results in order; every thread gets it.
__device__ __forceinline__ void zcd_block_max(double &d, int &i, double *sv, int *si)
{
    zcd_wave_max(d, i);
    const int w = threadIdx.x >> 6;
    __syncthreads();   // earlier readers of sv/si are done
    if ((threadIdx.x & 63) == 0) {
        sv[w] = d;
        si[w] = i;
    }
    __syncthreads();
    d = sv[0];
    i = si[0];
#pragma unroll
    for (int k = 1; k < 4; ++k) zcd_better(d, i, sv[k], si[k]);
}

// Largest entry of n_slots (d, idx) pairs, lowest idx on ties; every thread
// of the workgroup gets the result.
__device__ __forceinline__ void zcd_reduce(const Nom *slots, int n_slots, double &bd, int &bi,
                                           double *sv, int *si)
{
    double d = -INFINITY;
    int i = 0x7fffffff;
    for (int s = threadIdx.x; s < n_slots; s += 256) zcd_better(d, i, slots[s].d, slots[s].idx);
    zcd_block_max(d, i, sv, si);
    bd = d;
    bi = i;
}

__global__ __launch_bounds__(256) void k_zcd(const ZcdParams Z)
{
    __shared__ double sv[256];
    __shared__ int si[256];
    __shared__ double2 sacc[256];
    const int tid = threadIdx.x;
    const int g = blockIdx.x;
    const int R = Z.R, S = 256 / R;
    const int rl = tid % R, kl = tid / R;
    const int64_t n = Z.n;
    const int64_t r = (int64_t)g * R + rl;
    const bool own = r < n;
    unsigned int gen = 0;

    // initial diagonal and the first pivot
    double dmine = -INFINITY;
    if (own && kl == 0) {
        dmine = Z.A[r * n + r].x;
        Z.D[r] = dmine;
    }
    {
        double bd = (kl == 0) ? dmine : -INFINITY;
        int bi = (own && kl == 0) ? (int)r : 0x7fffffff;
        zcd_block_max(bd, bi, sv, si);
        if (tid == 0) {
            Z.part[g].d = bd;
            Z.part[g].idx = bi;
        }
    }
    if (!grid_barrier(Z.gs, Z.G, g, gen, Z.spin_limit)) {
        if (g == 0 && tid == 0) *Z.status = 5;
        return;
    }
    double d;
    int p;
    zcd_reduce(Z.part, Z.G, d, p, sv, si);
    const double floor_tol = (double)n * 0x1p-53 * fmax(d, 0.0);
    int64_t K = 0;
    for (;;) {
        // stop tests, identical in every workgroup
        int st = -1;
        if (n == 0 || d < Z.tau || (Z.tau <= 0.0 && d <= floor_tol)) st = 0;
        else if (K >= Z.max_vectors) st = 3;
        else if (!(d > 0.0) || !isfinite(d)) st = 4;
        if (st >= 0) {
            if (g == 0 && tid == 0) {
                *Z.status = st;
                *Z.n_vectors = K;
            }
            return;
        }
        if (g == 0 && tid == 0) Z.pivots[K] = p;
        // column K: this thread's share of sum_J L^J_r conj(L^J_p)
        double ar = 0.0, ai = 0.0;
        if (own) {
            const double2 *Lr = Z.L + r;
            const double2 *Lp = Z.L + p;
            int64_t J = kl;
            for (; J + 3 * S < K; J += 4 * S) {
                const double2 x0 = Lr[J * n], y0 = Lp[J * n];
                const double2 x1 = Lr[(J + S) * n], y1 = Lp[(J + S) * n];
                const double2 x2 = Lr[(J + 2 * S) * n], y2 = Lp[(J + 2 * S) * n];
                const double2 x3 = Lr[(J + 3 * S) * n], y3 = Lp[(J + 3 * S) * n];
                ar = fma(x0.x, y0.x, fma(x0.y, y0.y, ar));
                ai = fma(x0.y, y0.x, fma(-x0.x, y0.y, ai));
                ar = fma(x1.x, y1.x, fma(x1.y, y1.y, ar));
                ai = fma(x1.y, y1.x, fma(-x1.x, y1.y, ai));
                ar = fma(x2.x, y2.x, fma(x2.y, y2.y, ar));
                ai = fma(x2.y, y2.x, fma(-x2.x, y2.y, ai));
                ar = fma(x3.x, y3.x, fma(x3.y, y3.y, ar));
                ai = fma(x3.y, y3.x, fma(-x3.x, y3.y, ai));
            }
            for (; J < K; J += S) {
                const double2 x = Lr[J * n], y = Lp[J * n];
                ar = fma(x.x, y.x, fma(x.y, y.y, ar));
                ai = fma(x.y, y.x, fma(-x.x, y.y, ai));
            }
        }
        sacc[tid] = make_double2(ar, ai);
        __syncthreads();
        double dnew = -INFINITY;
        if (own && kl == 0) {
            double sr = 0.0, si_ = 0.0;
            for (int k = 0; k < S; ++k) {   // fixed order over the k-lanes
                sr += sacc[k * R + rl].x;
                si_ += sacc[k * R + rl].y;
            }
            const double2 a = Z.A[(int64_t)p * n + r];   // A(r, p) = conj(A(p, r))
            const double inv = 1.0 / sqrt(d);
            const double lr = (a.x - sr) * inv, li = (-a.y - si_) * inv;
            Z.L[K * n + r] = make_double2(lr, li);
            double dr = Z.D[r] - (lr * lr + li * li);
            if (r == p) dr = 0.0;
            Z.D[r] = dr;
            dnew = dr;
        }
        // largest updated residual of this workgroup's rows
        double bd = dnew;
        int bi = (own && kl == 0) ? (int)r : 0x7fffffff;
        zcd_block_max(bd, bi, sv, si);
        Nom *slots = Z.part + ((K + 1) & 1) * Z.G;
        if (tid == 0) {
            slots[g].d = bd;
            slots[g].idx = bi;
        }
        if (!grid_barrier(Z.gs, Z.G, g, gen, Z.spin_limit)) {
            if (g == 0 && tid == 0) {
                *Z.status = 5;
                *Z.n_vectors = K + 1;
            }
            return;
        }
        ++K;
        zcd_reduce(slots, Z.G, d, p, sv, si);
    }
}

__global__ void k_zcd_init(GridSync *gs, int32_t *status, int64_t *n_vectors)
{
    for (int i = threadIdx.x; i < kMaxGridBlocks * 16; i += blockDim.x) gs->arrive[i] = 0u;
    if (threadIdx.x == 0) {
        gs->release = 0u;
        gs->abort = 0u;
        *status = 0;
        *n_vectors = 0;
    }
}

}  // namespace cdk

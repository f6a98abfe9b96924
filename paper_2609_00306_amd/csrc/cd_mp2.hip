// Closed-shell second-order (MP2) energy from transformed Cholesky vectors.
//
// The CD-based MP2 of the paper (Secs. 5 and 7) first transforms the vectors
// to the molecular-orbital basis (the O(N^3 M) step, cd_transform with the
// occupied and the virtual coefficients) and then contracts them:
//     (ia|jb) = sum_P B[P][i][a] B[P][j][b],
//     e_ij    = sum_{ab} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b),
//     E       = sum_{ij} e_ij,   e_ji = e_ij
// (the energy expression is the textbook closed-shell one).
//
// One workgroup per (pair i <= j, virtual tile pair TA <= TB of 64 x 64):
// W1 = B_i(:, TA)^T B_j(:, TB) and, off the tile diagonal, W2 =
// B_i(:, TB)^T B_j(:, TA), both FP64 MFMA products over P (k-major operands,
// the shared gemm_tile engine).  When the last tile TB holds at most 48
// virtuals, both products take it as their row side with only as many 16-row
// tiles as it needs, which trims the matrix work spent on its zero padding.  The epilogue adds the terms of every ordered
// (a, b) with a in TA, b in TB and, off the diagonal, (b, a); a fixed-order
// reduction leaves one partial per workgroup.  Then one workgroup per pair
// adds its tile pairs, and one workgroup adds the pairs (i == j once, i < j
// twice).  Work items are laid out so that the tile pairs of one (i, j) run
// on one XCD and share B_i, B_j through its L2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "cd_mfma.hpp"

namespace cdk {

constexpr int MP2_TKC = 32;
using Mp2Stage = OperandStage<64, MP2_TKC, true>;

struct Mp2Params {
    const double *B;           // [max_vectors][O][V]
    int64_t max_vectors;
    const int64_t *n_vectors;  // [1]
    int32_t O, V;
    const double *eo, *ev;     // [O], [V]
    int32_t T, TP, NP;         // virtual tiles, tile pairs, occupied pairs
    int64_t per_xcd;           // work items per XCD slot
    double *partial;           // [NP][TP]
    double *pair_e;            // [NP]
    double *pair_out;          // optional [O][O]
    double *energy;            // [1]
    int32_t *status;           // [1]
};

// Upper-triangle index p = j (j + 1) / 2 + i, i <= j, back to (i, j).
__device__ __forceinline__ void tri_pair(int p, int &i, int &j)
{
    int jj = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while (jj * (jj + 1) / 2 > p) --jj;
    while ((jj + 1) * (jj + 2) / 2 <= p) ++jj;
    j = jj;
    i = p - jj * (jj + 1) / 2;
}

// Fixed-order sum of one value per thread of the 256-thread workgroup; the
// result is valid in thread 0.
__device__ __forceinline__ double block_sum_fixed(double v, double *s)
{
    const int tid = threadIdx.x;
    s[tid] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) s[tid] = s[tid] + s[tid + w];
        __syncthreads();
    }
    return s[0];
}

__global__ __launch_bounds__(256) void k_mp2_tiles(const Mp2Params Q)
{
    __shared__ double sStage[2 * Mp2Stage::kSize];   // operand staging; W2 afterwards
    __shared__ double sW1[64][65];
    __shared__ double sRed[256];
    const int tid = threadIdx.x;
    const int64_t g = blockIdx.x;
    const int64_t item = (g & 7) * Q.per_xcd + (g >> 3);
    const int64_t total = (int64_t)Q.NP * Q.TP;
    if (item >= total) return;
    const int p = (int)(item / Q.TP), tp = (int)(item % Q.TP);
    int i, j, TA, TB;
    tri_pair(p, i, j);
    tri_pair(tp, TA, TB);
    int64_t M = *Q.n_vectors;
    if (M < 0 || M > Q.max_vectors) M = 0;   // reported by k_mp2_total
    const int O = Q.O, V = Q.V;
    const int64_t ldP = (int64_t)O * V;
    const double *__restrict__ B = Q.B;
    double *sA = sStage;
    double *sB = sStage + Mp2Stage::kSize;
    double *sW2 = sStage;   // [64][64] once the second product is done
    const int lane = tid & 63, w = tid >> 6;

    // acc[r] = B_x(:, 64 tr + 16 r + .)^T B_y(:, 64 tc + 16 w + .), RT row tiles
    auto product = [&](int x, int tr, int y, int tc, auto &acc) {
        constexpr int RT = sizeof(acc) / sizeof(acc[0]);
        zero_acc(acc);
        gemm_tile<RT, MP2_TKC, true, true>(
            0, M,
            [&](int64_t k, int m) -> double {
                const int a = 64 * tr + m;
                return (a < V) ? B[k * ldP + (int64_t)x * V + a] : 0.0;
            },
            [&](int64_t k, int n) -> double {
                const int b = 64 * tc + n;
                return (b < V) ? B[k * ldP + (int64_t)y * V + b] : 0.0;
            },
            acc, sA, sB);
    };
    // acc element (row m, column n) -> W1[a][b] or W2[b][a] in LDS; 'swap' when
    // the product was formed with the tiles exchanged (rows from TB)
    auto store = [&](const auto &acc, double *dst, int ld, bool swap) {
        constexpr int RT = sizeof(acc) / sizeof(acc[0]);
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = 16 * r + mfma_row(lane, v), n = 16 * w + (lane & 15);
                if (swap) dst[n * ld + m] = acc[r][v];
                else dst[m * ld + n] = acc[r][v];
            }
    };
    // A last virtual tile with at most 48 virtuals in use is taken as the row
    // side of both products with ceil(used / 16) row tiles instead of 4: W1 is
    // then formed as W1^T = B_j(:, TB)^T B_i(:, TA) and stored transposed.
    auto short_pair = [&](auto rt_tag) {
        constexpr int RT = decltype(rt_tag)::value;
        f64x4 acc[RT];
        if (TA != TB) {
            product(j, TB, i, TA, acc);   // W1^T
            store(acc, &sW1[0][0], 65, true);
            product(i, TB, j, TA, acc);   // W2
            store(acc, sW2, 64, false);
        } else {
            product(i, TA, j, TB, acc);   // rows and columns both in the short tile
            store(acc, &sW1[0][0], 65, false);
        }
    };
    const int rt_tb = (TB == Q.T - 1) ? (V - 64 * TB + 15) / 16 : 4;
    if (rt_tb == 1) {
        short_pair(std::integral_constant<int, 1>{});
    } else if (rt_tb == 2) {
        short_pair(std::integral_constant<int, 2>{});
    } else if (rt_tb == 3) {
        short_pair(std::integral_constant<int, 3>{});
    } else {
        f64x4 acc[4];
        product(i, TA, j, TB, acc);
        store(acc, &sW1[0][0], 65, false);
        if (TA != TB) {
            product(i, TB, j, TA, acc);   // ends with a barrier: the staging is free
            store(acc, sW2, 64, false);
        }
    }
    __syncthreads();
    const double ei = Q.eo[i], ej = Q.eo[j];
    double s = 0.0;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int m = e >> 6, n = e & 63;
        const int a = 64 * TA + m, b = 64 * TB + n;
        if (a < V && b < V) {
            const double wab = sW1[m][n];
            const double wba = (TA == TB) ? sW1[n][m] : sW2[n * 64 + m];
            const double den = ei + ej - Q.ev[a] - Q.ev[b];
            s += wab * (2.0 * wab - wba) / den;
            if (TA != TB) s += wba * (2.0 * wba - wab) / den;
        }
    }
    const double tot = block_sum_fixed(s, sRed);
    if (tid == 0) Q.partial[item] = tot;
}

// e_ij of every pair: its tile pairs added in order.
__global__ __launch_bounds__(64) void k_mp2_pairs(const Mp2Params Q)
{
    const int p = blockIdx.x;
    if (threadIdx.x != 0 || p >= Q.NP) return;
    double s = 0.0;
    for (int t = 0; t < Q.TP; ++t) s += Q.partial[(int64_t)p * Q.TP + t];
    Q.pair_e[p] = s;
    if (Q.pair_out) {
        int i, j;
        tri_pair(p, i, j);
        Q.pair_out[(int64_t)i * Q.O + j] = s;
        Q.pair_out[(int64_t)j * Q.O + i] = s;
    }
}

// E = sum_i e_ii + 2 sum_{i<j} e_ij, in a fixed order; also the status word.
__global__ __launch_bounds__(256) void k_mp2_total(const Mp2Params Q)
{
    __shared__ double sRed[256];
    const int64_t M = *Q.n_vectors;
    const bool ok = M >= 0 && M <= Q.max_vectors;
    double s = 0.0;
    if (ok) {
        for (int p = threadIdx.x; p < Q.NP; p += 256) {
            int i, j;
            tri_pair(p, i, j);
            s += (i == j ? 1.0 : 2.0) * Q.pair_e[p];
        }
    }
    const double tot = block_sum_fixed(s, sRed);
    if (threadIdx.x == 0) {
        Q.energy[0] = ok ? tot : 0.0;
        Q.status[0] = ok ? 0 : 1;   // CD_ERR_INVALID_ARG: n_vectors outside [0, max_vectors]
    }
}

// Workspace doubles of one problem.
inline int64_t mp2_ws_doubles(int O, int V)
{
    const int64_t T = (V + 63) / 64, TP = T * (T + 1) / 2, NP = (int64_t)O * (O + 1) / 2;
    return NP * TP + NP + 1;
}

}  // namespace cdk

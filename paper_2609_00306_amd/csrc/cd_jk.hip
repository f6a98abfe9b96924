// Coulomb/exchange builds from the Cholesky vectors (paper Sec. 4.1: J costs
// O(N^2 M), K costs O(O N^2 M)) and the AO->MO transform of the vectors
// (Sec. 4.1, CASSCF; two-coefficient form of Sec. 6.2).
//
//   J_{mu nu} = sum_P L^P_{mu nu} V^P,  V^P = sum_{rho sigma} L^P_{rho sigma} D_{rho sigma},  D = C C^T
//   K_{mu nu} = sum_P sum_i X^P_{i mu} X^P_{i nu},  X^P_{i mu} = sum_sigma L^P_{mu sigma} C_{sigma i}
//   Lmo^P_{ab} = sum_{mu nu} C1_{mu a} L^P_{mu nu} C2_{nu b}
//
// L is packed over screened pairs (rows); a dense N x N row map unpacks it
// on the fly into the MFMA operand tiles.
#include <type_traits>

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

// w[r] = (2 - delta_{mu nu}) D_{mu nu} with D = C C^T (C [N][O]): the
// packed-row weight of the density, each entry taken straight from C (only the
// kept pairs' entries of D are needed).  16 lanes per row, lane j summing
// i = j, j + 16, ..; the 16 partial sums are added across the lanes.
__global__ __launch_bounds__(256) void k_drow(int64_t n_rows, const int64_t *__restrict__ row_pair,
                                              int O, const double *__restrict__ C,
                                              double *__restrict__ w)
{
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int j = threadIdx.x & 15;
    int mu = 0, nu = 0;
    double s = 0.0;
    if (r < n_rows) {
        unpack_pair(row_pair[r], mu, nu);
        const double *a = C + (int64_t)mu * O, *b = C + (int64_t)nu * O;
        for (int i = j; i < O; i += 16) s = fma(a[i], b[i], s);
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
    if (r < n_rows && j == 0) w[r] = (mu == nu) ? s : 2.0 * s;
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
    // four independent sums, so four loads per thread are in flight
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t r = threadIdx.x;
    for (; r + 768 < n_rows; r += 1024) {
        s0 = fma(row[r], w[r], s0);
        s1 = fma(row[r + 256], w[r + 256], s1);
        s2 = fma(row[r + 512], w[r + 512], s2);
        s3 = fma(row[r + 768], w[r + 768], s3);
    }
    for (; r < n_rows; r += 256) s0 = fma(row[r], w[r], s0);
    double s = (s0 + s1) + (s2 + s3);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) V[Pv] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

// J at row r = sum_P L[P][r] V[P]; written to both (mu,nu) and (nu,mu).
// 64 rows per workgroup, the vectors split over the 4 waves, combined in LDS.
__global__ __launch_bounds__(256) void k_jJ(const double *__restrict__ L, int64_t n_rows,
                                            const double *__restrict__ V,
                                            const int64_t *__restrict__ n_vectors,
                                            const int64_t *__restrict__ row_pair, int N,
                                            double *__restrict__ J)
{
    __shared__ double s_part[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * 64 + lane;
    const int64_t M = *n_vectors;
    // eight independent sums, so eight loads per lane are in flight
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (r < n_rows) {
        int64_t Pv = w;
        for (; Pv + 28 < M; Pv += 32) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                s[j] = fma(L[(Pv + 4 * j) * n_rows + r], V[Pv + 4 * j], s[j]);
        }
        for (; Pv < M; Pv += 4) s[0] = fma(L[Pv * n_rows + r], V[Pv], s[0]);
    }
    s_part[w][lane] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    __syncthreads();
    if (w == 0 && r < n_rows) {
        const double tot = (s_part[0][lane] + s_part[1][lane]) + (s_part[2][lane] + s_part[3][lane]);
        int mu, nu;
        unpack_pair(row_pair[r], mu, nu);
        J[(int64_t)mu * N + nu] = tot;
        J[(int64_t)nu * N + mu] = tot;
    }
}


// ---------------------------------------------------------------- sparse unpacking
// The unpacked vector Lt^P[mu][sigma] is nonzero only on kept pairs, so the
// half transform runs over each function's neighbour list (sigma with (mu,
// sigma) kept, ascending sigma) instead of all N sigma.  The vectors are
// first transposed to row-major LT[row][P] so that one row's M values are
// contiguous.

// LT[r][P] = L[P][r]  (64 x 64 tiles through LDS)
__global__ __launch_bounds__(256) void k_transpose(const double *__restrict__ L, int64_t n_rows,
                                                   const int64_t *__restrict__ n_vectors,
                                                   double *__restrict__ LT, int64_t ldt)
{
    __shared__ double t[64][65];
    const int64_t r0 = (int64_t)blockIdx.x * 64, p0 = (int64_t)blockIdx.y * 64;
    const int64_t M = *n_vectors;
    if (p0 >= M) return;
    // all 16 loads of a thread in flight before the first LDS write
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int e = threadIdx.x + 256 * j, pp = e >> 6, rr = e & 63;
        v[j] = (p0 + pp < M && r0 + rr < n_rows) ? L[(p0 + pp) * n_rows + r0 + rr] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int e = threadIdx.x + 256 * j;
        t[e >> 6][e & 63] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int e = threadIdx.x + 256 * j, rr = e >> 6, pp = e & 63;
        if (r0 + rr < n_rows && p0 + pp < M) LT[(r0 + rr) * ldt + p0 + pp] = t[pp][rr];
    }
}

// deg[mu] = number of kept pairs (mu, sigma) over all sigma; one wave per mu
__global__ __launch_bounds__(256) void k_nbr_count(const int32_t *__restrict__ rowof, int N,
                                                   int32_t *__restrict__ deg)
{
    const int mu = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (mu >= N) return;
    int c = 0;
    for (int s0 = 0; s0 < N; s0 += 64) {
        const int sg = s0 + lane;
        c += __popcll(__ballot(sg < N && rowof[(int64_t)mu * N + sg] >= 0));
    }
    if (lane == 0) deg[mu] = c;
}

// off[0..N]: exclusive prefix sum of deg (one workgroup)
__global__ __launch_bounds__(256) void k_scan_deg(const int32_t *__restrict__ deg, int N,
                                                  int64_t *__restrict__ off)
{
    __shared__ int64_t s[256];
    __shared__ int64_t base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int c0 = 0; c0 < N; c0 += 256) {
        const int i = c0 + threadIdx.x;
        const int64_t v = (i < N) ? deg[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const int64_t a = (threadIdx.x >= o) ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < N) off[i] = base + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 255) base += s[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[N] = base;
}

// neighbour lists in ascending sigma: nb_s = sigma, nb_r = row of (mu, sigma)
__global__ __launch_bounds__(256) void k_nbr_fill(const int32_t *__restrict__ rowof, int N,
                                                  const int64_t *__restrict__ off,
                                                  int32_t *__restrict__ nb_s,
                                                  int32_t *__restrict__ nb_r)
{
    const int mu = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (mu >= N) return;
    int64_t pos = off[mu];
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int s0 = 0; s0 < N; s0 += 64) {
        const int sg = s0 + lane;
        const int32_t r = (sg < N) ? rowof[(int64_t)mu * N + sg] : -1;
        const unsigned long long b = __ballot(r >= 0);
        if (r >= 0) {
            const int64_t q = pos + __popcll(b & below);
            nb_s[q] = sg;
            nb_r[q] = r;
        }
        pos += __popcll(b);
    }
}

// Half transform over neighbour lists (FP64 matrix cores):
//   Y[mu][P * ncol + i] = sum_{j in nbr(mu)} LT[r_j][P] C[sigma_j][i]
// OUT selects what is written: HALF_F64 the FP64 result, row mu at mu * ldy;
// HALF_BF16X3 the result split into three BF16 planes (split_bf16x3), plane p
// at Yp + p * plane: the operand of the 3 x BF16 exchange product, split once
// here instead of in every tile that reads it; HALF_F32 the result rounded to
// FP32 (the operand of the FP32 exchange product).  The last two forms are
// k-blocked (xb_index, ldy = the padded row count R), and a non-null Y64 also
// receives the FP64 value (row-major, row mu at mu * ldy64).
//
// k-blocked layout of the reduced-precision X: the k index (P * ncol + i) is
// cut into blocks of XB_K values, and block b holds the XB_K values of every
// row mu contiguously at (b R + mu) XB_K.  A k-step of the exchange product
// (one block, 128 rows) is then one contiguous run of memory instead of 128
// rows far apart.
constexpr int XB_K = 32;
__host__ __device__ __forceinline__ int64_t xb_index(int64_t mu, int64_t e, int64_t rows)
{
    return ((e / XB_K) * rows + mu) * XB_K + e % XB_K;
}

// x = b0 + b1 + b2 + O(2^-24 |x|): f = fp32(x), b0 = bf16(f), b1 = bf16(f - b0),
// b2 = bf16(f - b0 - b1), every rounding to nearest; the differences are exact
// in FP32 (each operand pair lies within a factor of two), so the split is
// plain FP32 arithmetic.  |x - f| <= 2^-24 |x| and the part past b2 is below
// 2^-27 |f|, both under the 2^-16 order the six products keep.
__device__ __forceinline__ void split_bf16x3(double x, __bf16 &b0, __bf16 &b1, __bf16 &b2)
{
    const float f = (float)x;
    b0 = (__bf16)f;
    const float r1 = f - (float)b0;
    b1 = (__bf16)r1;
    b2 = (__bf16)(r1 - (float)b1);
}

// Output forms of the half transform.
enum HalfOut { HALF_F64 = 0, HALF_BF16X3 = 1, HALF_F32 = 2 };

// A 512-thread workgroup covers 128 vectors P and 16 CT columns i of one
// function mu (CT = 10: all of them for ncol <= 160; CT = 4 for ncol <= 64),
// so each neighbour's LT row segment is read once per column range; wave w
// owns the 16 vectors 16 w and all CT column tiles.  Chunks of 16 neighbours
// go straight from memory into two LDS buffers one chunk ahead of the
// products (global_load_lds, 16-byte pieces gathered through the neighbour
// list staged in LDS; one barrier per chunk).  With 78 KB of LDS and at most
// 128 registers per lane two workgroups share a compute unit, so one's loads
// and stores overlap the other's products (three buffers and one workgroup per
// unit: 5.6 against 4.9 ms for the FP64 form on the 1200-function workload).  A part [k][128] from LT (rows
// padded to whole 128-vector tiles), B part [k][16 CT] from Cp, C copied with
// rows padded to whole column ranges and one extra zero row that the ragged
// last chunk reads past the list.  The 16-byte piece j of an odd row k is
// stored at j ^ 8.
constexpr int HS_P = 128;     // vectors per workgroup
constexpr int HS_TK = 16;     // neighbours per chunk
constexpr int HS_SEG = 512;   // neighbour-list entries staged in LDS at a time

// column tiles of the half transform for ncol columns
__host__ __device__ constexpr int hs_col_tiles(int ncol) { return (ncol <= 64) ? 4 : 10; }

template <int OUT, int CT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_half_sparse(const double *__restrict__ LT, int64_t ldt,
                                                     const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ nb_s,
                                                     const int32_t *__restrict__ nb_r,
                                                     const double *__restrict__ Cp, int ldc,
                                                     int zero_row, int ncol,
                                                     const int64_t *__restrict__ n_vectors,
                                                     void *__restrict__ Yv, int64_t ldy,
                                                     int64_t plane, double *__restrict__ Y64,
                                                     int64_t ldy64)
{
    constexpr int HS_C = 16 * CT;                 // columns per workgroup
    constexpr int kA = HS_TK * HS_P, kB = HS_TK * HS_C, kChunk = kA + kB;
    constexpr int kBL = kB / 128;                  // 16-byte-piece loads of B per chunk
    constexpr int kBW = (kBL + 7) / 8;             // per wave, waves < kBL % 8 one more
    static_assert(CT % 2 == 0, "whole 16-byte pieces per row pair");
    // two chunk buffers; after the products, the staged output planes
    __shared__ __align__(16) double sU[2 * kChunk];
    __shared__ int sNs[HS_SEG], sNr[HS_SEG];
    const int64_t M = *n_vectors;
    const int64_t p0 = (int64_t)blockIdx.x * HS_P;
    if (p0 >= M) return;
    const int n0 = blockIdx.y * HS_C;
    const int mu = blockIdx.z;
    const int64_t j0 = off[mu], deg = off[mu + 1] - j0;
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    f64x4 acc[CT];
    zero_acc(acc);
    auto swz = [&](int k, int col) -> int { return 2 * ((col >> 1) ^ (8 * (k & 1))) + (col & 1); };
    // B pieces of this lane: instruction v covers pieces [64 (8 v + w), +64) of
    // the chunk's [16][8 CT] piece array
    int bk[kBW], bj[kBW];
#pragma unroll
    for (int v = 0; v < kBW; ++v) {
        const int pc = 64 * (8 * v + w) + lane;
        bk[v] = pc / (HS_C / 2);
        bj[v] = 2 * ((pc % (HS_C / 2)) ^ (8 * (bk[v] & 1)));
    }
    for (int64_t seg = 0; seg < deg; seg += HS_SEG) {
        const int len = (int)min((int64_t)HS_SEG, deg - seg);
        __syncthreads();
        // past the list: the zero row of Cp against a valid LT row
        for (int e = tid; e < HS_SEG; e += 512) {
            sNs[e] = (e < len) ? nb_s[j0 + seg + e] : zero_row;
            sNr[e] = nb_r[j0 + seg + min(e, len - 1)];
        }
        __syncthreads();
        const int nch = (len + HS_TK - 1) / HS_TK;
        auto load_chunk = [&](int c, int buf) __attribute__((always_inline)) {
            double *st = sU + buf * kChunk;
            const int kc = c * HS_TK;
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int k = 8 * v + w;   // A row k is this instruction's KB
                const double *src = LT + (int64_t)sNr[kc + k] * ldt + p0 + 2 * (lane ^ (8 * (k & 1)));
                lds_dma16(src, (lds_void *)(st + 128 * k));
            }
#pragma unroll
            for (int v = 0; v < kBW; ++v) {
                if (8 * v + w < kBL) {
                    const double *src = Cp + (int64_t)sNs[kc + bk[v]] * ldc + n0 + bj[v];
                    lds_dma16(src, (lds_void *)(st + kA + 128 * (8 * v + w)));
                }
            }
        };
        if (nch > 0) load_chunk(0, 0);
        int buf = 0;
        for (int c = 0; c < nch; ++c) {
            // own pieces of chunk c landed, then a barrier: every wave's pieces
            // of chunk c are in, and every wave is done with the buffer that
            // chunk c + 1 refills (chunk c - 1's); chunk c + 1 loads while
            // chunk c is multiplied
            wait_vmcnt<0>();
            lds_barrier();
            if (c + 1 < nch) load_chunk(c + 1, buf ^ 1);
            const double *sA = sU + buf * kChunk, *sB = sA + kA;
            buf ^= 1;
#pragma unroll
            for (int s = 0; s < HS_TK / 4; ++s) {
                const int k = 4 * s + (lane >> 4);
                const double a = sA[k * HS_P + swz(k, 16 * w + (lane & 15))];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                    const double bv = sB[k * HS_C + swz(k, 16 * ct + (lane & 15))];
                    acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[ct], 0, 0, 0);
                }
            }
        }
    }
    // acc[ct][v]: vector p0 + 16 w + mfma_row(lane, v), column n0 + 16 ct + lane % 16
    if constexpr (OUT != HALF_F64) if (gridDim.y == 1) {
        // All columns in one workgroup: its outputs are the contiguous range
        // e in [p0 ncol, (p0 + np) ncol), which starts on a k-block (p0 is a
        // multiple of 128).  The planes go through LDS in e order (each value
        // split once), 64 vectors at a time, and out as 16-byte runs, eight
        // (FP32) or four (BF16) of which fill a block row, instead of 2- or
        // 4-byte stores scattered over the blocks.
        using OT = typename std::conditional<OUT == HALF_F32, float, __bf16>::type;
        constexpr int G = 16 / (int)sizeof(OT);
        constexpr int NPL = (OUT == HALF_F32) ? 1 : 3;
        constexpr int PH = HS_P / 2;      // vectors per staged half (waves 0-3, then 4-7)
        constexpr int PS = PH * HS_C;     // values per staged plane of a half
        static_assert(NPL * PS * sizeof(OT) <= sizeof(sU), "a half's planes fit in LDS");
        const int np = (int)min((int64_t)HS_P, M - p0);
        OT *T = reinterpret_cast<OT *>(sU);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // the half's outputs: e in [(p0 + PH h) ncol, (p0 + min(np, PH (h + 1))) ncol),
            // again starting on a k-block (PH ncol is a multiple of XB_K)
            const int nh = min(np - PH * h, PH);
            if (nh <= 0) break;
            const int len = nh * ncol;
            const int64_t e0 = (p0 + PH * h) * ncol;
            __syncthreads();   // every wave is done with the chunk buffers / the last half
            if ((w >> 2) == h) {
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int P = 16 * (w & 3) + mfma_row(lane, v);
                        const int n = 16 * ct + (lane & 15);
                        if (P < nh && n < ncol) {
                            if constexpr (OUT == HALF_F32) {
                                T[P * ncol + n] = (float)acc[ct][v];
                            } else {
                                __bf16 b0, b1, b2;
                                split_bf16x3(acc[ct][v], b0, b1, b2);
                                T[P * ncol + n] = b0;
                                T[PS + P * ncol + n] = b1;
                                T[2 * PS + P * ncol + n] = b2;
                            }
                        }
                    }
            }
            __syncthreads();
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) {
                OT *out = static_cast<OT *>(Yv) + pl * plane;
                const OT *Tp = T + pl * PS;
                for (int i = G * tid; i < len; i += G * 512) {
                    if (i + G <= len) {
                        *reinterpret_cast<uint4 *>(out + xb_index(mu, e0 + i, ldy)) =
                            *reinterpret_cast<const uint4 *>(Tp + i);
                    } else {
                        for (int j = i; j < len; ++j) out[xb_index(mu, e0 + j, ldy)] = Tp[j];
                    }
                }
            }
        }
        const int64_t e0 = p0 * ncol;
        if (Y64) {   // the FP64 value as well (C^T L C)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int P = 16 * w + mfma_row(lane, v);
                    const int n = 16 * ct + (lane & 15);
                    if (P < np && n < ncol) Y64[(int64_t)mu * ldy64 + e0 + P * ncol + n] = acc[ct][v];
                }
        }
        return;
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t P = p0 + 16 * w + mfma_row(lane, v);
            const int n = n0 + 16 * ct + (lane & 15);
            if (P >= M || n >= ncol) continue;
            const double x = acc[ct][v];
            const int64_t e = P * ncol + n;
            if (OUT == HALF_F64) {
                static_cast<double *>(Yv)[(int64_t)mu * ldy + e] = x;
            } else if (OUT == HALF_F32) {
                static_cast<float *>(Yv)[xb_index(mu, e, ldy)] = (float)x;
                if (Y64) Y64[(int64_t)mu * ldy64 + e] = x;   // the FP64 value as well (C^T L C)
            } else {
                __bf16 b0, b1, b2;
                split_bf16x3(x, b0, b1, b2);
                __bf16 *out = static_cast<__bf16 *>(Yv) + xb_index(mu, e, ldy);
                out[0] = b0;
                out[plane] = b1;
                out[2 * plane] = b2;
                if (Y64) Y64[(int64_t)mu * ldy64 + e] = x;   // the FP64 value as well (C^T L C)
            }
        }
}


// Work item of a split-k exchange product launched as a 1-D grid of
// pairs x nsplit workgroups (nsplit a multiple of 8).  Workgroups are dealt to
// the 8 XCDs round robin, so workgroup g runs on XCD g % 8; giving every k-split
// to one XCD (all tile pairs of split s on XCD s % 8, dispatched together)
// lets the pairs that read the same rows of X share that XCD's L2, and each
// k-chunk of X comes from memory once per split instead of once per pair.
__device__ __forceinline__ void syrk_tile_split(int N, int nsplit, int &t, int &s)
{
    const int T = (N + 63) / 64, pairs = T * (T + 1) / 2;
    const int g = blockIdx.x, xcd = g & 7, j = g >> 3;
    s = xcd + 8 * (j / pairs);
    t = j % pairs;
    (void)nsplit;
}

// Partial K from row-major X (row mu holds the M * ncol values X^P_{i mu}):
//   Kp[s][mu][nu] = sum_{k in slab s} X[mu][k] X[nu][k]   (lower tile pairs)
// A 256-thread workgroup owns a 64 x 64 tile pair; wave w the 32 x 32 quarter
// (rows 32 (w / 2), columns 32 (w % 2)) as 2 x 2 accumulators of the 16x16x4
// FP64 instruction.  k-chunks of 32 values of the 128 rows (both sides: 32 KB)
// go straight from memory into two LDS buffers one chunk ahead of the products
// (global_load_lds, 16-byte pieces, 8 per lane per chunk; one barrier per
// chunk); LDS rows are 256 bytes, unpadded, with the k-pair index XORed with
// row % 16.  64 KB of LDS: two workgroups per compute unit.  (Chunks of 16 in
// a three-buffer ring, three workgroups per unit, made the 1200-function J/K
// build 2 ms slower; chunks of 32 in three buffers, one workgroup per unit,
// 6 ms slower.)  It serves the sizes where 128 x 128 tiles (k_syrk_rows128)
// would pad much more: N = 400 takes 448 rows in 64 x 64 tiles, 512 in 128 x
// 128 ones, and the diagonal tiles compute less of the upper triangle.
constexpr int XR_TK = 32;    // k per chunk
constexpr int XR_NST = 2;    // chunk buffers (loads run XR_NST - 1 chunks ahead)
constexpr int XR_STAGE = 128 * XR_TK;          // doubles per chunk
constexpr int XR_LOADS = XR_STAGE / 2 / 256;   // 16-byte pieces per lane per chunk
constexpr int XR_RPW = 64 / (XR_TK / 2);       // rows one wave's 64 pieces cover
static_assert(XR_TK == 16 || XR_TK == 32, "chunk of 16 or 32 values");
static_assert(XR_NST == 2 || XR_NST == 3, "two or three chunk buffers");
// stored k-pair slot of k-pair g in row r: g ^ xr_swz(r), so the 16 rows read
// at one k-pair by a quarter-wave fall on different banks
__device__ __forceinline__ int xr_swz(int r) { return (XR_TK == 16) ? ((r >> 1) & 7) : (r & 15); }
__global__ __launch_bounds__(256) void k_syrk_rows(const double *__restrict__ X, int64_t ldx,
                                                   int N, const int64_t *__restrict__ n_vectors,
                                                   int ncol, int nsplit, double *__restrict__ Kp)
{
    __shared__ __align__(16) double sX[XR_NST * XR_STAGE];
    int t, s;
    syrk_tile_split(N, nsplit, t, s);
    int tm = 0;
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    const int tn = t - tm * (tm + 1) / 2;
    const int64_t nk = *n_vectors * ncol;
    int64_t per = (nk + nsplit - 1) / nsplit;
    per = (per + XR_TK - 1) / XR_TK * XR_TK;
    const int64_t kb = s * per;
    const int64_t ke = (kb + per < nk) ? kb + per : nk;
    const int m0 = tm * 64, n0 = tn * 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // piece v of this lane: LDS row r = XR_RPW (4 v + w) + lane / (XR_TK / 2)
    // (rows 0..63 the A side m0.., 64..127 the B side n0..; rows past N read
    // row N - 1), slot lane % (XR_TK / 2), which holds k-pair
    // slot ^ xr_swz(r) of that row
    int64_t goff[XR_LOADS];
#pragma unroll
    for (int v = 0; v < XR_LOADS; ++v) {
        const int r = XR_RPW * (4 * v + w) + lane / (XR_TK / 2);
        const int grow = min((r < 64) ? m0 + r : n0 + r - 64, N - 1);
        goff[v] = (int64_t)grow * ldx + 2 * ((lane % (XR_TK / 2)) ^ xr_swz(r));
    }
    // a full chunk straight into LDS; a partial last chunk through registers
    // with the values past ke set to zero
    auto load_chunk = [&](double *st, int64_t k0) __attribute__((always_inline)) {
        if (k0 + XR_TK <= ke) {
#pragma unroll
            for (int v = 0; v < XR_LOADS; ++v)
                lds_dma16(X + k0 + goff[v], (lds_void *)(st + 128 * (4 * v + w)));
        } else {
            for (int e = tid; e < XR_STAGE; e += 256) {
                const int r = e / XR_TK, k = e % XR_TK;
                const int grow = min((r < 64) ? m0 + r : n0 + r - 64, N - 1);
                st[r * XR_TK + 2 * ((k >> 1) ^ xr_swz(r)) + (k & 1)] =
                    (k0 + k < ke) ? X[(int64_t)grow * ldx + k0 + k] : 0.0;
            }
        }
    };
    // operands of this lane at k-step q: row r with r % 16 = lane % 16,
    // k = 4 q + lane / 16, i.e. k-pair 2 q + lane / 32, element (lane / 16) % 2
    const int lr = lane & 15, sw = xr_swz(lr), hi = lane >> 5, el = (lane >> 4) & 1;
    const int ar = 32 * (w >> 1) + lr, br = 64 + 32 * (w & 1) + lr;
    f64x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    auto mma_chunk = [&](const double *S) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < XR_TK / 4; ++q) {
            const int col = 2 * ((2 * q + hi) ^ sw) + el;
            const double a0 = S[ar * XR_TK + col], a1 = S[(ar + 16) * XR_TK + col];
            const double b0 = S[br * XR_TK + col], b1 = S[(br + 16) * XR_TK + col];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    };
    // chunk c: its own loads landed (those of the next XR_NST - 2 chunks may
    // stay in flight), a barrier (every wave's pieces of chunk c are in, and
    // every wave is done with the buffer that chunk c + XR_NST - 1 refills), the
    // loads of chunk c + XR_NST - 1, then the products of chunk c
    const int64_t nch = (ke > kb) ? (ke - kb + XR_TK - 1) / XR_TK : 0;
#pragma unroll
    for (int c = 0; c < XR_NST - 1; ++c)
        if (c < nch) load_chunk(sX + c * XR_STAGE, kb + c * XR_TK);
    int buf = 0;
    for (int64_t c = 0; c < nch; ++c) {
        if (XR_NST == 3 && c + 1 < nch) wait_vmcnt<XR_LOADS>();
        else wait_vmcnt<0>();
        lds_barrier();
        if (c + XR_NST - 1 < nch)
            load_chunk(sX + ((buf == 0) ? XR_NST - 1 : buf - 1) * XR_STAGE, kb + (c + XR_NST - 1) * XR_TK);
        mma_chunk(sX + buf * XR_STAGE);
        buf = (buf == XR_NST - 1) ? 0 : buf + 1;
    }
    double *out = Kp + (int64_t)s * N * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + 32 * (w >> 1) + 16 * i + mfma_row(lane, e);
                const int n = n0 + 32 * (w & 1) + 16 * j + lr;
                if (m < N && n < N) out[(int64_t)m * N + n] = acc[i][j][e];
            }
}


// The same partial K over lower 128 x 128 tile pairs: wave w owns the 64 x 64
// quarter (rows 64 (w / 2), columns 64 (w % 2)) as 4 x 4 accumulators, so each
// operand read from LDS feeds four products.  k-chunks of 16 values of the 256
// rows (both sides: 32 KB) go straight into two LDS buffers one chunk ahead
// (global_load_lds, 8 pieces per lane per chunk); LDS rows are 128 bytes with
// the k-pair index XORed with (row / 2) % 8.  64 KB of LDS: two workgroups per
// compute unit.  Workgroup g runs on XCD g % 8; its j = g / 8 -th item is tile
// pair j % pairs of split 8 (j / pairs) + g % 8.
constexpr int XQ_TK = 16;
constexpr int XQ_STAGE = 256 * XQ_TK;          // doubles per chunk
constexpr int XQ_LOADS = XQ_STAGE / 2 / 256;   // 16-byte pieces per lane per chunk (8)
__global__ __launch_bounds__(256) void k_syrk_rows128(const double *__restrict__ X, int64_t ldx,
                                                      int N, const int64_t *__restrict__ n_vectors,
                                                      int ncol, int pairs, int nsplit,
                                                      double *__restrict__ Kp)
{
    __shared__ __align__(16) double sX[2 * XQ_STAGE];
    const int g = blockIdx.x, j = g >> 3, t = j % pairs, s = 8 * (j / pairs) + (g & 7);
    int tm = 0;
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    const int tn = t - tm * (tm + 1) / 2;
    const int64_t nk = *n_vectors * ncol;
    int64_t per = (nk + nsplit - 1) / nsplit;
    per = (per + XQ_TK - 1) / XQ_TK * XQ_TK;
    const int64_t kb = s * per;
    const int64_t ke = (kb + per < nk) ? kb + per : nk;
    const int m0 = tm * 128, n0 = tn * 128;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // piece v of this lane: LDS row r = 8 (4 v + w) + lane / 8 (rows 0..127 the
    // A side m0.., 128..255 the B side n0..; rows past N read row N - 1), slot
    // lane % 8, which holds k-pair (lane % 8) ^ ((r / 2) % 8) of that row
    int64_t goff[XQ_LOADS];
#pragma unroll
    for (int v = 0; v < XQ_LOADS; ++v) {
        const int r = 8 * (4 * v + w) + (lane >> 3);
        const int grow = min((r < 128) ? m0 + r : n0 + r - 128, N - 1);
        goff[v] = (int64_t)grow * ldx + 2 * ((lane & 7) ^ ((r >> 1) & 7));
    }
    // a full chunk straight into LDS
    auto load_chunk = [&](double *st, int64_t k0) __attribute__((always_inline)) {
#pragma unroll
        for (int v = 0; v < XQ_LOADS; ++v)
            lds_dma16(X + k0 + goff[v], (lds_void *)(st + 128 * (4 * v + w)));
    };
    // a partial last chunk through registers, the values past ke set to zero
    auto load_tail = [&](double *st, int64_t k0) __attribute__((always_inline)) {
        for (int e = tid; e < XQ_STAGE; e += 256) {
            const int r = e / XQ_TK, k = e % XQ_TK;
            const int grow = min((r < 128) ? m0 + r : n0 + r - 128, N - 1);
            st[r * XQ_TK + 2 * ((k >> 1) ^ ((r >> 1) & 7)) + (k & 1)] =
                (k0 + k < ke) ? X[(int64_t)grow * ldx + k0 + k] : 0.0;
        }
    };
    const int lr = lane & 15, sw = (lr >> 1) & 7, hi = lane >> 5, el = (lane >> 4) & 1;
    const int ar = 64 * (w >> 1) + lr, br = 128 + 64 * (w & 1) + lr;
    f64x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[i][jj] = f64x4{0.0, 0.0, 0.0, 0.0};
    // a wave whose 64 rows or 64 columns all lie past N (the padding of the
    // last tile) issues no products: the other workgroup on its compute unit
    // gets the matrix unit
    const bool idle = m0 + 64 * (w >> 1) >= N || n0 + 64 * (w & 1) >= N;
    auto mma_chunk = [&](const double *S) __attribute__((always_inline)) {
        if (idle) return;
#pragma unroll
        for (int q = 0; q < XQ_TK / 4; ++q) {
            const int col = 2 * ((2 * q + hi) ^ sw) + el;
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = S[(ar + 16 * i) * XQ_TK + col];
                b[i] = S[(br + 16 * i) * XQ_TK + col];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    acc[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[jj], acc[i][jj], 0, 0, 0);
        }
    };
    // the full chunks in the loop (no other path inside it), then the partial
    // last chunk, if any
    const int64_t nfull = (ke > kb) ? (ke - kb) / XQ_TK : 0;
    const bool tail = ke > kb + nfull * XQ_TK;
    if (nfull > 0) load_chunk(sX, kb);
    int buf = 0;
    for (int64_t c = 0; c < nfull; ++c) {
        wait_vmcnt<0>();
        lds_barrier();
        if (c + 1 < nfull) load_chunk(sX + (buf ^ 1) * XQ_STAGE, kb + (c + 1) * XQ_TK);
        mma_chunk(sX + buf * XQ_STAGE);
        buf ^= 1;
    }
    if (tail) {
        wait_vmcnt<0>();
        lds_barrier();   // every wave is done with the buffer the tail refills
        load_tail(sX + buf * XQ_STAGE, kb + nfull * XQ_TK);
        lds_barrier();
        mma_chunk(sX + buf * XQ_STAGE);
    }
    double *out = Kp + (int64_t)s * N * N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + 64 * (w >> 1) + 16 * i + mfma_row(lane, e);
                const int n = n0 + 64 * (w & 1) + 16 * jj + lr;
                if (m < N && n < N) out[(int64_t)m * N + n] = acc[i][jj][e];
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

// Second half of the transform as one wide product over all vectors:
//   O[a][c] = sum_mu C1[mu][a] Y[mu][c],   c = P q + b,   Lmo[P][a][b] = O[a][c]
// (Y from k_half_sparse with C2, row mu holding the M q values of that
// function).  Treating the vectors' columns as one long dimension pads only
// the a side to the tile (O = 150 takes 160 rows) instead of both sides of
// every vector's p x q block.
//
// A 512-thread workgroup covers 16 RA rows a (all of them for p <= 160) and
// 128 columns c; wave w owns the 16 columns 16 w and all RA row tiles, so Y,
// the large operand, is read exactly once over the grid.  k-chunks of 16
// functions go straight from memory into two LDS buffers one chunk ahead of
// the products (global_load_lds, 16-byte pieces, one barrier per chunk); at
// 72 KB of LDS and at most 128 registers two workgroups share a compute unit
// (5.35 -> 5.2 ms on the 1200-function workload against three buffers and one
// workgroup per unit):
//   A part: [k][16 RA] from C1p, C1 copied with its rows padded to whole
//           workgroup row ranges and to a whole number of chunks (zeros);
//   B part: [k][128] from Y, whose rows are padded to whole 128-column tiles.
// In both, the 16-byte piece j of an odd row k is stored at j ^ 8 (RA even),
// so the two rows a half-wave reads lie on different bank halves.  Rows of Y
// past N are read as row N - 1 against zero rows of C1p; columns past M q are
// never stored.
constexpr int TR_TK = 16;

// C1p[mu][a] = C1[mu][a] for mu < N, a < p, else 0   (rows of ld doubles)
__global__ void k_pack_c1(const double *__restrict__ C1, int N, int p, int rows, int ld,
                          double *__restrict__ C1p)
{
    const int64_t total = (int64_t)rows * ld;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int mu = (int)(e / ld), a = (int)(e % ld);
        C1p[e] = (mu < N && a < p) ? C1[(int64_t)mu * p + a] : 0.0;
    }
}

template <int RA>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_tr2w(const double *__restrict__ Y, int64_t ldy, int N,
                                              const double *__restrict__ C1p, int ldc, int p, int q,
                                              const int64_t *__restrict__ n_vectors,
                                              double *__restrict__ Lmo)
{
    static_assert(RA % 2 == 0 && RA <= 10, "row tiles: even, at most 10");
    constexpr int AL = 16 * RA;                 // A row length (doubles)
    constexpr int kA = TR_TK * AL, kB = TR_TK * 128, kChunk = kA + kB;
    constexpr int kAP = kA / 128;               // 16-byte-piece loads of A per chunk (RA + RA/4..)
    constexpr int kAL = kAP / 8, kAX = kAP % 8; // per wave, one more for waves < kAX
    __shared__ __align__(16) double sU[2 * kChunk];
    const int64_t ncol = *n_vectors * q;
    const int64_t c0 = (int64_t)blockIdx.x * 128;
    if (c0 >= ncol) return;
    const int a0 = blockIdx.y * AL;
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nch = (N + TR_TK - 1) / TR_TK;

    // B pieces: instruction v of this wave fills row k = 8 v + w of the chunk;
    // lane l's stored piece l holds column pair l ^ (8 (k % 2))
    const double *ysrc[2];
    int yrow[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        const int k = 8 * v + w;
        yrow[v] = k;
        ysrc[v] = Y + c0 + 2 * (lane ^ (8 * (k & 1)));
    }
    // A pieces: instruction i = 8 v + w covers pieces [64 i, 64 i + 64) of the
    // chunk's [16][AL / 2] piece array
    int aoff[kAL + 1];
#pragma unroll
    for (int v = 0; v <= kAL; ++v) {
        const int pc = 64 * (8 * v + w) + lane, k = pc / (AL / 2), j = pc % (AL / 2);
        aoff[v] = k * ldc + a0 + 2 * (j ^ (8 * (k & 1)));
    }
    auto load_chunk = [&](int c, int buf) __attribute__((always_inline)) {
        double *st = sU + buf * kChunk;
        const int kc = c * TR_TK;
        const double *a = C1p + (int64_t)kc * ldc;
#pragma unroll
        for (int v = 0; v <= kAL; ++v) {
            const int i = 8 * v + w;
            if (v < kAL || w < kAX) lds_dma16(a + aoff[v], (lds_void *)(st + 128 * i));
        }
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int64_t row = min(kc + yrow[v], N - 1);
            lds_dma16(ysrc[v] + row * ldy, (lds_void *)(st + kA + 128 * (8 * v + w)));
        }
    };
    f64x4 acc[RA];
    zero_acc(acc);
    // operand LDS indices: A[m][k] at k AL + swz(16 r + m), B[k][n] at k 128 + swz(16 w + n)
    const int m = lane & 15, kq = lane >> 4;
    auto swz = [&](int k, int col) -> int { return 2 * ((col >> 1) ^ (8 * (k & 1))) + (col & 1); };
    if (nch > 0) load_chunk(0, 0);
    int buf = 0;
    for (int c = 0; c < nch; ++c) {
        // own pieces of chunk c landed, then a barrier: every wave's pieces of
        // chunk c are in, and every wave is done with the buffer that chunk
        // c + 1 refills; chunk c + 1 loads while chunk c is multiplied
        wait_vmcnt<0>();
        lds_barrier();
        if (c + 1 < nch) load_chunk(c + 1, buf ^ 1);
        const double *sA = sU + buf * kChunk, *sB = sA + kA;
        buf ^= 1;
#pragma unroll
        for (int s = 0; s < TR_TK / 4; ++s) {
            const int k = 4 * s + kq;
            const double b = sB[k * 128 + swz(k, 16 * w + m)];
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                const double av = sA[k * AL + swz(k, 16 * r + m)];
                acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b, acc[r], 0, 0, 0);
            }
        }
    }
    const int64_t c = c0 + 16 * w + m;
    if (c < ncol) {
        const int64_t P = c / q, b = c % q;
        double *out = Lmo + P * (int64_t)p * q + b;
#pragma unroll
        for (int r = 0; r < RA; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = a0 + 16 * r + mfma_row(lane, v);
                if (a < p) out[(int64_t)a * q] = acc[r][v];
            }
    }
}

}  // namespace cdk

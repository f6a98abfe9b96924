// FP64 matrix-core tile for gfx950: one 256-thread workgroup computes a
// 64 x 64 block  acc[m][n] = sum_k A(k, m) B(k, n)  with both operands
// "k-major" (for a fixed k, m or n is the fast index), staged through LDS in
// k-chunks of 16.  Waves are arranged 2 x 2, each owning a 32 x 32 quarter as
// 2 x 2 tiles of v_mfma_f64_16x16x4f64.
//
// Operand/result lane layout of the 16x16x4 FP64 instruction (wave64):
//   A (16 x 4):  lane l holds A[m = l % 16][k = l / 16]
//   B (4 x 16):  lane l holds B[k = l / 16][n = l % 16]
//   D (16 x 16): lane l, element v holds D[m = 4 v + l / 16][n = l % 16]
// (the result layout was read back on gfx950 with a one-MFMA probe)
#pragma once
#include <hip/hip_runtime.h>

namespace cdk {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int TK = 16;    // k-chunk staged in LDS
constexpr int TM = 64;    // tile rows (m)
constexpr int TN = 64;    // tile cols (n)

struct TileAcc {
    f64x4 c[2][2];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) c[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
};

// sA, sB: LDS buffers of TK*TM doubles each.  la(k, m) / lb(k, n) return the
// operand for absolute k and tile-relative m / n (returning 0 outside).
template <class LoadA, class LoadB>
__device__ __forceinline__ void mfma_tile_f64(int64_t kbeg, int64_t kend, LoadA la, LoadB lb,
                                              TileAcc &acc, double *sA, double *sB)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wm = (w >> 1) * 32;
    const int wn = (w & 1) * 32;
    for (int64_t k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
        for (int u = 0; u < (TK * TM) / 256; ++u) {
            int e = tid + 256 * u;
            int kk = e >> 6;
            int mm = e & 63;
            int64_t k = k0 + kk;
            sA[e] = (k < kend) ? la(k, mm) : 0.0;
            sB[e] = (k < kend) ? lb(k, mm) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < TK; ks += 4) {
            int kr = ks + (lane >> 4);
            double a0 = sA[kr * TM + wm + (lane & 15)];
            double a1 = sA[kr * TM + wm + 16 + (lane & 15)];
            double b0 = sB[kr * TN + wn + (lane & 15)];
            double b1 = sB[kr * TN + wn + 16 + (lane & 15)];
            acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.c[0][0], 0, 0, 0);
            acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.c[0][1], 0, 0, 0);
            acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.c[1][0], 0, 0, 0);
            acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.c[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
}

// Row of the 16 x 16 result held by element v of 'lane'.
__device__ __forceinline__ int mfma_row(int lane, int v) { return 4 * v + (lane >> 4); }

// Write the accumulator into an LDS tile sT[m * ldt + n].
__device__ __forceinline__ void tile_to_lds(const TileAcc &acc, double *sT, int ldt)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wm = (w >> 1) * 32;
    const int wn = (w & 1) * 32;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int m = wm + 16 * i + mfma_row(lane, v);
                int n = wn + 16 * j + (lane & 15);
                sT[m * ldt + n] = acc.c[i][j][v];
            }
}

}  // namespace cdk

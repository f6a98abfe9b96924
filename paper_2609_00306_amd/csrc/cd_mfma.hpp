// FP64 matrix-core GEMM engine for gfx950.
//
// One 256-thread workgroup (4 waves) computes a (16 RT) x 64 block
//     acc[m][n] = sum_k A(k, m) B(k, n)
// Wave w owns the 16 columns [16 w, 16 w + 16) and all RT row tiles, one
// v_mfma_f64_16x16x4f64 accumulator per row tile.  Operands are staged through
// LDS in k-chunks of TKC; the next chunk is loaded into registers while the
// current one is multiplied (software pipelining), so global-memory latency
// overlaps the matrix work.  Each operand is either "k-major" (for fixed k the
// m/n index is contiguous in memory) or "k-contiguous" (for fixed m/n the k
// index is contiguous); the global-load mapping follows the contiguous index
// so every load is coalesced.
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

// Row of the 16 x 16 result held by element v of 'lane'.
__device__ __forceinline__ int mfma_row(int lane, int v) { return 4 * v + (lane >> 4); }

template <int ROWS, int TKC, bool KMAJ, int NT = 256>
struct OperandStage {
    // LDS footprint in doubles; NT threads share the loads
    static constexpr int kStride = KMAJ ? ROWS : (TKC + 1);
    static constexpr int kSize = KMAJ ? TKC * ROWS : ROWS * (TKC + 1);
    static constexpr int kPerThread = (ROWS * TKC + NT - 1) / NT;

    // element e of a chunk -> (k, m), following the contiguous index
    __device__ static __forceinline__ void coord(int e, int &k, int &m)
    {
        if (KMAJ) {
            k = e / ROWS;
            m = e % ROWS;
        } else {
            m = e / TKC;
            k = e % TKC;
        }
    }
    __device__ static __forceinline__ int lds_index(int k, int m)
    {
        return KMAJ ? k * ROWS + m : m * (TKC + 1) + k;
    }
    template <class LD>
    __device__ static __forceinline__ void fetch(LD ld, int64_t k0, int64_t kend, double (&r)[kPerThread])
    {
#pragma unroll
        for (int u = 0; u < kPerThread; ++u) {
            int e = threadIdx.x + NT * u;
            int k, m;
            coord(e, k, m);
            r[u] = (e < ROWS * TKC && k0 + k < kend) ? ld(k0 + k, m) : 0.0;
        }
    }
    __device__ static __forceinline__ void put(double *s, const double (&r)[kPerThread])
    {
#pragma unroll
        for (int u = 0; u < kPerThread; ++u) {
            int e = threadIdx.x + NT * u;
            if (e < ROWS * TKC) {
                int k, m;
                coord(e, k, m);
                s[lds_index(k, m)] = r[u];
            }
        }
    }
};

// acc[r] += A(k, 16 r + .) B(k, 16 w + .)  for k in [kbeg, kend), all RT row
// tiles (rows a caller does not need read zeros from its loader; updating every
// accumulator unconditionally keeps them out of control flow, which the
// register allocator otherwise answers with accumulator copies).  la(k, m),
// lb(k, n) return the operands (k absolute, m in [0, 16 RT), n in [0, 64));
// loads with k >= kend are not issued.  sA, sB: LDS of OperandStage<..>::kSize
// doubles.
template <int RT, int TKC, bool AK, bool BK, class LA, class LB>
__device__ __forceinline__ void gemm_tile(int64_t kbeg, int64_t kend, LA la, LB lb,
                                          f64x4 (&acc)[RT], double *sA, double *sB)
{
    using SA = OperandStage<16 * RT, TKC, AK>;
    using SB = OperandStage<64, TKC, BK>;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    if (kbeg >= kend) return;
    double ra[SA::kPerThread], rb[SB::kPerThread];
    SA::fetch(la, kbeg, kend, ra);
    SB::fetch(lb, kbeg, kend, rb);
    for (int64_t k0 = kbeg; k0 < kend; k0 += TKC) {
        SA::put(sA, ra);
        SB::put(sB, rb);
        __syncthreads();
        if (k0 + TKC < kend) {
            SA::fetch(la, k0 + TKC, kend, ra);
            SB::fetch(lb, k0 + TKC, kend, rb);
        }
#pragma unroll
        for (int ks = 0; ks < TKC; ks += 4) {
            const int kk = ks + (lane >> 4);
            const double b = sB[SB::lds_index(kk, 16 * w + (lane & 15))];
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const double a = sA[SA::lds_index(kk, 16 * r + (lane & 15))];
                acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[r], 0, 0, 0);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- split-k form
// Wave-parallel product for short, tall operands: every wave owns whole
// k-chunks of 16 (chunk c goes to wave c % 4), stages them in its own LDS
// region and keeps a full (16 RT) x 64 accumulator, so the four waves run
// four independent load/multiply pipelines with no workgroup-wide barrier
// inside the k loop.  Both operands are rows of one row-major matrix 'base'
// (k contiguous, rows 16-byte aligned): A rows for the 16 RT output rows, B
// rows for the 64 output columns.  Each lane loads one 16-byte piece of 8
// different rows per chunk (8 lanes cover a row's 128 bytes), from row
// offsets it keeps in registers, so no index lookup precedes a load.  The
// partial products are summed across waves by wave_sum_to_lds().
template <int RT>
struct SplitK {
    static constexpr int TKC = 16;
    static constexpr int kRows = 16 * RT;
    static constexpr int kLd = TKC + 2;                          // 16-byte aligned LDS rows
    static constexpr int kWaveDoubles = (kRows + 64) * kLd;     // LDS per wave
    static constexpr int kNA = kRows / 8;                        // A rows per lane
    static constexpr int kNB = 64 / 8;                           // B rows per lane

    // Row handled by this lane in load slot u (A or B).
    __device__ static __forceinline__ int row_of(int u) { return ((threadIdx.x & 63) >> 3) + 8 * u; }

    template <int NR>
    __device__ static __forceinline__ void fetch_rows(const double *__restrict__ base,
                                                      const int64_t (&off)[NR], int64_t k0,
                                                      int64_t kend, double2 (&v)[NR])
    {
        const int64_t k = k0 + 2 * (threadIdx.x & 7);
        if (k0 + TKC <= kend) {
#pragma unroll
            for (int u = 0; u < NR; ++u)
                v[u] = (off[u] >= 0) ? *reinterpret_cast<const double2 *>(base + off[u] + k)
                                     : double2{0.0, 0.0};
        } else {
#pragma unroll
            for (int u = 0; u < NR; ++u) {
                v[u].x = (off[u] >= 0 && k < kend) ? base[off[u] + k] : 0.0;
                v[u].y = (off[u] >= 0 && k + 1 < kend) ? base[off[u] + k + 1] : 0.0;
            }
        }
    }

    template <int NR>
    __device__ static __forceinline__ void put_rows(double *s, const double2 (&v)[NR])
    {
        const int c = 2 * (threadIdx.x & 7);
#pragma unroll
        for (int u = 0; u < NR; ++u) *reinterpret_cast<double2 *>(s + row_of(u) * kLd + c) = v[u];
    }

    // aoff[u] / boff[u]: element offset of the A / B row row_of(u) in 'base', or -1
    // for a row that is absent (read as zeros).  k runs over [0, kend).
    __device__ static __forceinline__ void run(int64_t kend, int rt, const double *__restrict__ base,
                                               const int64_t (&aoff)[kNA], const int64_t (&boff)[kNB],
                                               f64x4 (&acc)[RT][4], double *sWaves)
    {
        const int lane = threadIdx.x & 63;
        const int w = threadIdx.x >> 6;
        double *sAw = sWaves + w * kWaveDoubles;
        double *sBw = sAw + kRows * kLd;
        double2 va[kNA], vb[kNB];
        const int64_t nch = (kend + TKC - 1) / TKC;
        if (w >= nch) return;
        fetch_rows(base, aoff, (int64_t)w * TKC, kend, va);
        fetch_rows(base, boff, (int64_t)w * TKC, kend, vb);
        for (int64_t c = w; c < nch; c += 4) {
            put_rows(sAw, va);
            put_rows(sBw, vb);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (c + 4 < nch) {
                fetch_rows(base, aoff, (c + 4) * TKC, kend, va);
                fetch_rows(base, boff, (c + 4) * TKC, kend, vb);
            }
#pragma unroll
            for (int ks = 0; ks < TKC; ks += 4) {
                const int kk = ks + (lane >> 4);
                double b[4];
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) b[ct] = sBw[(16 * ct + (lane & 15)) * kLd + kk];
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    if (r < rt) {   // uniform
                        const double a = sAw[(16 * r + (lane & 15)) * kLd + kk];
#pragma unroll
                        for (int ct = 0; ct < 4; ++ct)
                            acc[r][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[ct],
                                                                               acc[r][ct], 0, 0, 0);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }

    // Each wave stores its accumulators into its own region,
    // sOut[w * region + m * 65 + n] (m < 16 rt): no read-modify-write, the
    // reader sums the four regions.  Must be called by the whole workgroup;
    // sOut may alias the wave regions.
    __device__ static __forceinline__ void wave_store_partials(const f64x4 (&acc)[RT][4], int rt,
                                                               double *sOut, int region)
    {
        const int lane = threadIdx.x & 63;
        const int w = threadIdx.x >> 6;
        double *o = sOut + w * region;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            if (r < rt) {
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        o[(16 * r + mfma_row(lane, v)) * 65 + 16 * ct + (lane & 15)] = acc[r][ct][v];
            }
        }
        __syncthreads();
    }

    // Sum the four waves' accumulators into sOut[m * 65 + n] (m < 16 rt).
    // Must be called by the whole workgroup; sOut may alias the wave regions.
    __device__ static __forceinline__ void wave_sum_to_lds(const f64x4 (&acc)[RT][4], int rt,
                                                           double *sOut)
    {
        const int lane = threadIdx.x & 63;
        const int w = threadIdx.x >> 6;
        __syncthreads();
        for (int step = 0; step < 4; ++step) {
            if (w == step) {
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    if (r < rt) {
#pragma unroll
                        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const int m = 16 * r + mfma_row(lane, v);
                                const int n = 16 * ct + (lane & 15);
                                double &o = sOut[m * 65 + n];
                                o = (step == 0) ? acc[r][ct][v] : o + acc[r][ct][v];
                            }
                    }
                }
            }
            __syncthreads();
        }
    }
};

// ---------------------------------------------------------------- LDS staging
typedef __attribute__((address_space(3))) void lds_void;

// Workgroup barrier that orders LDS only: a fence restricted to LDS, so the
// memory loads in flight (the next steps' pieces) need not complete first, as
// they would at __syncthreads().  The pieces loaded straight into LDS are
// waited for explicitly (wait_vmcnt) before the barrier.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One 16-byte piece per lane from global memory straight into LDS: lane l
// writes bytes [16 l, 16 l + 16) of the wave's KB at 'lds' (wave-uniform, it
// goes to M0).  Written as inline assembly (no output registers: the load
// writes LDS only) so that the compiler, which drains every load of this kind
// in flight before any LDS read, leaves the prefetch alone; the caller waits
// for the pieces explicitly (wait_vmcnt: loads complete in issue order) before
// the barrier that publishes them.
__device__ __forceinline__ void lds_dma16(const void *g, lds_void *lds)
{
    const uint32_t m0 = (uint32_t)(uintptr_t)lds;
    asm volatile("global_load_lds_dwordx4 %0, off" : : "v"(g), "{m0}"(m0) : "memory");
}

// One 4-byte piece per lane straight into LDS: lane l writes bytes [4 l, 4 l + 4)
// of the wave's 256 bytes at 'lds' (wave-uniform, it goes to M0); otherwise as
// lds_dma16.  Needs only 4-byte alignment of 'g'.
__device__ __forceinline__ void lds_dma4(const void *g, lds_void *lds)
{
    const uint32_t m0 = (uint32_t)(uintptr_t)lds;
    asm volatile("global_load_lds_dword %0, off" : : "v"(g), "{m0}"(m0) : "memory");
}

// s_waitcnt with only vmcnt limited (expcnt and lgkmcnt at their maxima); the
// 6-bit count is split over bits 3:0 and 15:14 of the immediate
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt immediate");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int RT>
__device__ __forceinline__ void zero_acc(f64x4 (&acc)[RT])
{
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = f64x4{0.0, 0.0, 0.0, 0.0};
}

// Visit every accumulator element: f(m, n, value) with m in [0, 16 RT), n in [0, 64).
template <int RT, class F>
__device__ __forceinline__ void for_each_acc(const f64x4 (&acc)[RT], int rt_active, F f)
{
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        if (r < rt_active) {
#pragma unroll
            for (int v = 0; v < 4; ++v) f(16 * r + mfma_row(lane, v), 16 * w + (lane & 15), acc[r][v]);
        }
    }
}

}  // namespace cdk

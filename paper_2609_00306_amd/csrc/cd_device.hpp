// Device-side building blocks shared by the library's kernels (gfx950).
//
// Integrals over normalised s-type Gaussians g(r) = (2a/pi)^{3/4} exp(-a|r-A|^2).
// For a pair (mu nu): p = a_mu + a_nu, P = (a_mu A_mu + a_nu A_nu)/p,
// E = N_mu N_nu exp(-a_mu a_nu/p |A_mu - A_nu|^2).  The paper evaluates ERIs
// with the McMurchie-Davidson scheme (Sec. 7); for s functions it reduces to
//   (ab|cd) = 2 pi^{5/2} / (p q sqrt(p+q)) E_ab E_cd F0(T),  T = pq/(p+q)|P-Q|^2,
// with F0(T) = (1/2) sqrt(pi/T) erf(sqrt T), F0(0) = 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdk {

constexpr double kPi = 3.14159265358979323846;
constexpr double kPi52x2 = 34.986836655249725;     // 2 pi^{5/2}
constexpr double kSqrtPiHalf = 0.88622692545275801; // sqrt(pi)/2

// One screened row: pair centre, exponent sum and c = E/p.
struct __align__(64) RowRec {
    double x, y, z, p;   // product centre P and exponent p
    double c;            // E / p
    double d1;           // (mu nu|mu nu)
    double pad0, pad1;
};

__device__ __forceinline__ void unpack_pair(int64_t pq, int &mu, int &nu)
{
    double s = sqrt(8.0 * (double)pq + 1.0);
    int64_t m = (int64_t)((s - 1.0) * 0.5);
    while (m * (m + 1) / 2 > pq) --m;
    while ((m + 1) * (m + 2) / 2 <= pq) ++m;
    mu = (int)m;
    nu = (int)(pq - m * (m + 1) / 2);
}

__device__ __forceinline__ RowRec make_row(const double *__restrict__ xyz,
                                           const double *__restrict__ alpha, int mu, int nu)
{
    double a = alpha[mu], b = alpha[nu];
    double ax = xyz[3 * mu], ay = xyz[3 * mu + 1], az = xyz[3 * mu + 2];
    double bx = xyz[3 * nu], by = xyz[3 * nu + 1], bz = xyz[3 * nu + 2];
    double p = a + b;
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    double r2 = dx * dx + dy * dy + dz * dz;
    double na = pow(2.0 * a / kPi, 0.75);
    double nb = pow(2.0 * b / kPi, 0.75);
    double e = na * nb * exp(-a * b / p * r2);
    RowRec R;
    R.x = (a * ax + b * bx) / p;
    R.y = (a * ay + b * by) / p;
    R.z = (a * az + b * bz) / p;
    R.p = p;
    R.c = e / p;
    // T = 0: 2 pi^{5/2} E^2 / (p^2 sqrt(2p))
    R.d1 = kPi52x2 * R.c * R.c / sqrt(2.0 * p);
    R.pad0 = 0.0;
    R.pad1 = 0.0;
    return R;
}

// F0(T) = int_0^1 exp(-T t^2) dt
__device__ __forceinline__ double boys0(double T)
{
    if (T < 1e-8) return 1.0 - T * (1.0 / 3.0);
    double x = sqrt(T);
    return kSqrtPiHalf * erf(x) / x;
}

__device__ __forceinline__ double eri(const RowRec &a, double bx, double by, double bz,
                                      double bp, double bc)
{
    double s = a.p + bp;
    double dx = a.x - bx, dy = a.y - by, dz = a.z - bz;
    double r2 = dx * dx + dy * dy + dz * dz;
    double T = a.p * bp / s * r2;
    return kPi52x2 * a.c * bc / sqrt(s) * boys0(T);
}

__device__ __forceinline__ double eri(const RowRec &a, const RowRec &b)
{
    return eri(a, b.x, b.y, b.z, b.p, b.c);
}

// ---------------------------------------------------------------- grid barrier
// Barrier for a cooperative launch (all workgroups co-resident) without a
// contended counter: every workgroup publishes its arrival in its own
// 64-byte slot, workgroup 0 polls all slots in parallel (one thread per
// slot) and then opens the next generation with a single flag that the
// others poll.  Stores are agent-scope releases and polls agent-scope
// acquires, so everything written before the barrier is visible after it
// (across XCDs).  Every wait is bounded: after 'spin_limit' polls the
// workgroup gives up, raises 'abort' and reports false.
constexpr int kMaxGridBlocks = 256;

struct GridSync {
    unsigned int release;
    unsigned int abort;
    unsigned int pad[14];
    unsigned int arrive[kMaxGridBlocks * 16];   // one 64-byte slot per workgroup
};

// Polls with relaxed agent-scope loads (no cache invalidation per poll) and
// takes one agent-scope acquire fence once the value is seen.
__device__ __forceinline__ bool spin_until_eq(unsigned int *addr, unsigned int want,
                                              unsigned int *abort_flag, unsigned int spin_limit)
{
    unsigned int spins = 0;
    while (__hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > spin_limit ||
            __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// 'nblocks' workgroups take part; 'me' is this workgroup's index among them.
__device__ __forceinline__ bool grid_barrier(GridSync *gs, unsigned int nblocks, unsigned int me,
                                             unsigned int &gen_local, unsigned int spin_limit)
{
    __shared__ int s_ok;
    const unsigned int want = gen_local + 1u;
    gen_local = want;
    if (threadIdx.x == 0) s_ok = 1;
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(&gs->arrive[me * 16], want, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    if (me == 0) {
        for (unsigned int i = threadIdx.x; i < nblocks; i += blockDim.x)
            if (!spin_until_eq(&gs->arrive[i * 16], want, &gs->abort, spin_limit)) s_ok = 0;
        __syncthreads();
        if (threadIdx.x == 0 && s_ok)
            __hip_atomic_store(&gs->release, want, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else if (threadIdx.x == 0) {
        if (!spin_until_eq(&gs->release, want, &gs->abort, spin_limit)) s_ok = 0;
    }
    __syncthreads();
    return s_ok != 0;
}

// ---------------------------------------------------------------- ordering
// Pivot order: larger residual first, lower row index on ties.
struct Nom {
    double d;
    int32_t idx;
    int32_t pad;
};

__device__ __forceinline__ bool nom_before(double da, int ia, double db, int ib)
{
    // evaluated without short-circuit branches (bitwise on the two tests)
    return (da > db) | ((da == db) & (ia < ib));
}

// In-place bitonic sort of n (power of two, 32 <= n <= 1024) entries in LDS
// into pivot order, by the whole 256-thread block; entries at 'valid' and past
// it are not read and sort as fillers (-inf, largest index).  Thread t holds entries
// 4t .. 4t+3 in registers: partners at distance 1 and 2 are in the same
// thread, at distance 4 .. 255 in another lane of the same wave (exchanged
// with DPP, swizzles or lane permutes chosen per stage at compile time, no
// barrier), and only at distance 256 and 512 in another wave (through LDS, two
// barriers per stage); up to 256 entries are sorted by wave 0 alone.  Only d
// and idx are sorted; 'pad' is left undefined.  Must be called by all threads
// of the block after the entries are visible to all of them.
__device__ __forceinline__ void nom_cmpx(double &d, int &x, double od, int ox, int e, int p, int k)
{
    const bool asc = (e & k) == 0;               // this run goes in pivot order
    const bool me_first = nom_before(d, x, od, ox);
    const bool take = ((e < p) == asc) != me_first;
    d = take ? od : d;
    x = take ? ox : x;
}

// Compare-exchange of register entries a < b (compile-time indices) of one
// thread; e is the element index of entry a.
__device__ __forceinline__ void nom_cmpx_regs(double (&d)[4], int (&x)[4], int a, int b, int e, int k)
{
    const bool asc = (e & k) == 0;
    const bool swap = asc != nom_before(d[a], x[a], d[b], x[b]);
    const double da = d[a], db = d[b];
    const int xa = x[a], xb = x[b];
    d[a] = swap ? db : da;
    x[a] = swap ? xb : xa;
    d[b] = swap ? da : db;
    x[b] = swap ? xa : xb;
}

// Value of lane (l ^ m) for a compile-time lane mask m < 64: DPP quad
// permutes for m = 1, 2, swizzles inside 32-lane halves for m = 4, 8, 16, and a
// lane permute for m = 32.
template <int M>
__device__ __forceinline__ int lane_xor(int v)
{
    if constexpr (M == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);
    else if constexpr (M == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);
    else if constexpr (M == 4 || M == 8 || M == 16) return __builtin_amdgcn_ds_swizzle(v, (M << 10) | 0x1f);
    else return __shfl_xor(v, M, 64);
}

template <int M>
__device__ __forceinline__ double lane_xor_d(double v)
{
    return __hiloint2double(lane_xor<M>(__double2hiint(v)), lane_xor<M>(__double2loint(v)));
}

// One bitonic stage (run length K, partner distance J, both compile-time) on
// the four register entries of every thread (entries 4t .. 4t+3).
template <int K, int J>
__device__ __forceinline__ void nom_stage(double (&d)[4], int (&x)[4], Nom *s)
{
    const int tid = threadIdx.x;
    if constexpr (J == 1) {
        nom_cmpx_regs(d, x, 0, 1, 4 * tid, K);
        nom_cmpx_regs(d, x, 2, 3, 4 * tid + 2, K);
    } else if constexpr (J == 2) {
        nom_cmpx_regs(d, x, 0, 2, 4 * tid, K);
        nom_cmpx_regs(d, x, 1, 3, 4 * tid + 1, K);
    } else if constexpr (J < 256) {
        double od[4];
        int ox[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {   // all exchanges in flight before any compare
            od[r] = lane_xor_d<J / 4>(d[r]);
            ox[r] = lane_xor<J / 4>(x[r]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = 4 * tid + r;
            nom_cmpx(d[r], x[r], od[r], ox[r], e, e ^ J, K);
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            s[4 * tid + r].d = d[r];
            s[4 * tid + r].idx = x[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = 4 * tid + r, p = e ^ J;
            nom_cmpx(d[r], x[r], s[p].d, s[p].idx, e, p, K);
        }
    }
}

// All stages of run length K (partner distances K/2 .. 1).
template <int K, int J>
__device__ __forceinline__ void nom_merge(double (&d)[4], int (&x)[4], Nom *s)
{
    nom_stage<K, J>(d, x, s);
    if constexpr (J > 1) nom_merge<K, J / 2>(d, x, s);
}

// Run lengths K .. KMAX, stopping at the first one above n (uniform).
template <int K, int KMAX>
__device__ __forceinline__ void nom_sort_from(double (&d)[4], int (&x)[4], Nom *s, int n)
{
    if (K > n) return;
    nom_merge<K, K / 2>(d, x, s);
    if constexpr (K < KMAX) nom_sort_from<2 * K, KMAX>(d, x, s, n);
}

__device__ __forceinline__ void block_sort_noms(Nom *s, int n, int valid)
{
    const int tid = threadIdx.x;
    // up to 256 entries live in wave 0 alone (no barrier inside the sort)
    const bool active = n > 256 || tid < 64;
    double d[4];
    int x[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = 4 * tid + r;
        d[r] = (e < valid) ? s[e].d : -INFINITY;
        x[r] = (e < valid) ? s[e].idx : 0x7fffffff;
    }
    if (n > 256) nom_sort_from<2, 1024>(d, x, s, n);
    else if (active) nom_sort_from<2, 256>(d, x, s, n);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = 4 * tid + r;
        if (e < n) {
            s[e].d = d[r];
            s[e].idx = x[r];
        }
    }
    __syncthreads();
}

// Wave-wide (64 lanes) maximum of an unsigned value with DPP max steps; the
// result is read from lane 63.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v)
{
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Lowest lane holding the largest positive value (values <= 0, -inf and NaN
// never win), or -1 if no lane holds one; 'best' receives the value.  The bit
// pattern of a positive double orders like an unsigned integer, so the maximum
// is taken on the high word; only if several lanes share that high word is
// the low word compared among them.  Exact, with 32-bit DPP steps only.
__device__ __forceinline__ int wave_argmax_pos(double v, double &best)
{
    const unsigned long long key = (v > 0.0) ? (unsigned long long)__double_as_longlong(v) : 0ull;
    const unsigned hi = (unsigned)(key >> 32), lo = (unsigned)key;
    const unsigned mh = wave_max_u32(hi);
    const unsigned long long th = __ballot(hi == mh && key != 0ull);
    if (th == 0ull) {
        best = 0.0;
        return -1;
    }
    unsigned long long tie = th;
    if (th & (th - 1)) {   // several lanes share the high word
        const unsigned ml = wave_max_u32(hi == mh ? lo : 0u);
        tie = __ballot(hi == mh && lo == ml && key != 0ull);
    }
    const int bl = (int)__ffsll((long long)tie) - 1;
    const int blo = __builtin_amdgcn_readlane((int)lo, bl);
    best = __longlong_as_double((long long)(((unsigned long long)mh << 32) | (unsigned)blo));
    return bl;
}

// Wave-wide (64 lanes) minimum of an unsigned value with DPP min steps; the
// result is read from lane 63.
__device__ __forceinline__ unsigned wave_min_u32(unsigned v)
{
    const int id = -1;   // 0xffffffff, the identity of the minimum
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x111, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x112, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x114, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x118, 0xf, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x142, 0xa, 0xf, false));
    v = min(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x143, 0xc, 0xf, false));
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// The lane holding the first entry in pivot order (larger d, then lower idx)
// among lanes whose d is positive or +inf; -1 if there is none.  Exact: the
// maximum of d is taken on its bit pattern (high word, then low word among
// ties), and equal d are broken by the minimum idx.
__device__ __forceinline__ int wave_pick_first(double d, int idx)
{
    const unsigned long long key = (d > 0.0) ? (unsigned long long)__double_as_longlong(d) : 0ull;
    const unsigned hi = (unsigned)(key >> 32), lo = (unsigned)key;
    const unsigned mh = wave_max_u32(hi);
    unsigned long long tie = __ballot(hi == mh && key != 0ull);
    if (tie == 0ull) return -1;
    if (tie & (tie - 1)) {
        const unsigned ml = wave_max_u32(hi == mh ? lo : 0u);
        tie = __ballot(hi == mh && lo == ml && key != 0ull);
        if (tie & (tie - 1)) {
            const bool mine = (tie >> (threadIdx.x & 63)) & 1ull;
            const unsigned mi = wave_min_u32(mine ? (unsigned)idx : 0xffffffffu);
            tie = __ballot(mine && (unsigned)idx == mi);
        }
    }
    return (int)__ffsll((long long)tie) - 1;
}

// 1 / sqrt(x) for a positive normal x: the hardware estimate refined by two
// Newton steps y <- y + y (1/2 - (x/2) y^2), accurate to about one unit in the
// last place.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = fma(y, fma(-h * y, y, 0.5), y);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}

// Wave-wide (64 lanes) selection of the lane holding the first entry in pivot order.
__device__ __forceinline__ void wave_best(double &d, int &idx, int &lane_of)
{
    int lane = threadIdx.x & 63;
    lane_of = lane;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double od = __shfl_xor(d, off, 64);
        int oi = __shfl_xor(idx, off, 64);
        int ol = __shfl_xor(lane_of, off, 64);
        if (nom_before(od, oi, d, idx)) {
            d = od;
            idx = oi;
            lane_of = ol;
        }
    }
}

}  // namespace cdk

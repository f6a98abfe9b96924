// Kernels of the threshold-truncated, fully pivoted Cholesky decomposition of
// the ERI matrix over composite pair indices (paper Sec. 2; the two-step
// organisation of Sec. 3 with exact pivoting).
//
//   setup   : pair table, diagonal D1 = (r|r), screening, compaction of the
//             rows and of the "active" rows (D1 >= tau: the only possible
//             pivots, since D never increases -- Sec. 3; with restricted
//             candidates, Sec. 6.2, also both functions flagged).
//   step 1  : one persistent cooperative kernel selects the pivots on the
//             active rows only.  Per batch it takes the top-q active rows as
//             candidates, forms their Schur-complement columns in one pass
//             (Eq. (subtr) for q pivots at once), then every workgroup
//             factors the q x q candidate block redundantly, accepting the
//             next candidate only while it is provably the global argmax:
//             it must come before (in pivot order) every row outside the
//             candidate set, which is bounded by the first row left out.
//             Accepted pivots are applied to all active rows (D update of
//             Eq. (diag)).  Two grid barriers per batch instead of one per
//             pivot; the pivot sequence is exactly that of Sec. 2.
//   step 2  : every row's vector elements from the pivot-row block
//             (Sec. 3, Eq. CVsLT): a blocked forward substitution with
//             the ERIs (r|P_K) generated in the tile epilogue, FP64 MFMA.
#include "cd_device.hpp"
#include "cd_mfma.hpp"
#include "cd_kernels.hpp"

namespace cdk {

// ---------------------------------------------------------------- setup
__global__ __launch_bounds__(256) void k_diag_all(int N, const double *__restrict__ xyz,
                                                  const double *__restrict__ alpha,
                                                  int64_t npairs, double *__restrict__ D1all,
                                                  unsigned long long *d1max_bits)
{
    __shared__ double s_max[4];
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double d = 0.0;
    if (k < npairs) {
        int mu, nu;
        unpack_pair(k, mu, nu);
        RowRec R = make_row(xyz, alpha, mu, nu);
        d = R.d1;
        D1all[k] = d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off, 64));
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3]));
        atomicMax(d1max_bits, (unsigned long long)__double_as_longlong(m));
    }
}

// keep: the row survives screening; act: it may become a pivot (D1 >= tau
// and, with restricted candidates, both functions flagged -- Sec. 6.2).
__device__ __forceinline__ void row_flags(double d1, double mx, double schwarz, double tau,
                                          bool cand, bool &keep, bool &act)
{
    keep = sqrt(d1 * mx) >= schwarz;
    act = keep && cand && (d1 >= tau);
}

// Row k may be a pivot under the per-function flags (null: every row).
__device__ __forceinline__ bool pair_is_candidate(int64_t k, const uint8_t *__restrict__ pivot_fn)
{
    if (!pivot_fn) return true;
    int mu, nu;
    unpack_pair(k, mu, nu);
    return pivot_fn[mu] != 0 && pivot_fn[nu] != 0;
}

// Per-256-pair block counts of kept and active rows.
__global__ __launch_bounds__(256) void k_count(int64_t npairs, const double *__restrict__ D1all,
                                               const unsigned long long *d1max_bits,
                                               double schwarz, double tau,
                                               const uint8_t *__restrict__ pivot_fn,
                                               int32_t *__restrict__ cnt_rows,
                                               int32_t *__restrict__ cnt_act)
{
    __shared__ int s_c[2][4];
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mx = __longlong_as_double((long long)*d1max_bits);
    bool keep = false, act = false;
    if (k < npairs) row_flags(D1all[k], mx, schwarz, tau, pair_is_candidate(k, pivot_fn), keep, act);
    unsigned long long bk = __ballot(keep);
    unsigned long long ba = __ballot(act);
    if ((threadIdx.x & 63) == 0) {
        s_c[0][threadIdx.x >> 6] = __popcll(bk);
        s_c[1][threadIdx.x >> 6] = __popcll(ba);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt_rows[blockIdx.x] = s_c[0][0] + s_c[0][1] + s_c[0][2] + s_c[0][3];
        cnt_act[blockIdx.x] = s_c[1][0] + s_c[1][1] + s_c[1][2] + s_c[1][3];
    }
}

// Exclusive prefix sums of the block counts (one workgroup); totals at the end.
__global__ __launch_bounds__(256) void k_scan(int32_t nblk, const int32_t *__restrict__ cnt_rows,
                                              const int32_t *__restrict__ cnt_act,
                                              int64_t *__restrict__ off_rows,
                                              int64_t *__restrict__ off_act,
                                              int64_t *__restrict__ totals)
{
    __shared__ int64_t s_a[256], s_b[256];
    __shared__ int64_t s_base[2];
    if (threadIdx.x == 0) {
        s_base[0] = 0;
        s_base[1] = 0;
    }
    __syncthreads();
    for (int32_t c0 = 0; c0 < nblk; c0 += 256) {
        int32_t i = c0 + threadIdx.x;
        int64_t a = (i < nblk) ? cnt_rows[i] : 0;
        int64_t b = (i < nblk) ? cnt_act[i] : 0;
        s_a[threadIdx.x] = a;
        s_b[threadIdx.x] = b;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            int64_t va = (threadIdx.x >= off) ? s_a[threadIdx.x - off] : 0;
            int64_t vb = (threadIdx.x >= off) ? s_b[threadIdx.x - off] : 0;
            __syncthreads();
            s_a[threadIdx.x] += va;
            s_b[threadIdx.x] += vb;
            __syncthreads();
        }
        if (i < nblk) {
            off_rows[i] = s_base[0] + s_a[threadIdx.x] - a;
            off_act[i] = s_base[1] + s_b[threadIdx.x] - b;
        }
        __syncthreads();
        if (threadIdx.x == 255) {
            s_base[0] += s_a[255];
            s_base[1] += s_b[255];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        totals[0] = s_base[0];
        totals[1] = s_base[1];
    }
}

// Compaction: rows in ascending packed order, active rows in ascending row order.
__global__ __launch_bounds__(256) void k_scatter(
    int N, const double *__restrict__ xyz, const double *__restrict__ alpha, int64_t npairs,
    const double *__restrict__ D1all, const unsigned long long *d1max_bits, double schwarz,
    double tau, const uint8_t *__restrict__ pivot_fn, const int64_t *__restrict__ off_rows, const int64_t *__restrict__ off_act,
    int64_t n_cap, int64_t na_cap, int64_t *__restrict__ row_pair, RowRec *__restrict__ rows, int32_t *__restrict__ act_row,
    double *__restrict__ D_act, int32_t *__restrict__ pivot_of_row)
{
    __shared__ int s_c[2][4];
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mx = __longlong_as_double((long long)*d1max_bits);
    bool keep = false, act = false;
    if (k < npairs) row_flags(D1all[k], mx, schwarz, tau, pair_is_candidate(k, pivot_fn), keep, act);
    unsigned long long bk = __ballot(keep);
    unsigned long long ba = __ballot(act);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) {
        s_c[0][w] = __popcll(bk);
        s_c[1][w] = __popcll(ba);
    }
    __syncthreads();
    int64_t pk = off_rows[blockIdx.x], pa = off_act[blockIdx.x];
    for (int i = 0; i < w; ++i) {
        pk += s_c[0][i];
        pa += s_c[1][i];
    }
    pk += __popcll(bk & below);
    pa += __popcll(ba & below);
    if (keep && pk < n_cap) {
        int mu, nu;
        unpack_pair(k, mu, nu);
        row_pair[pk] = k;
        rows[pk] = make_row(xyz, alpha, mu, nu);
        pivot_of_row[pk] = -1;
        if (act && pa < na_cap) {
            act_row[pa] = (int32_t)pk;
            D_act[pa] = D1all[k];
        }
    }
}

// ---------------------------------------------------------------- step 1
constexpr int QMAX = 64;       // candidate batch size
constexpr int CNOM = 4;        // nominations per workgroup
constexpr int SMAX = 256;      // active rows per workgroup
constexpr int NOMSORT = 1024;  // union capacity (workgroups * CNOM)
constexpr int S1_MAXG = NOMSORT / CNOM;
using S1K = SplitK<3>;         // candidate-column product: 48 rows per pass, k-chunks of 16
// all-row solve
constexpr int S2_NB = 128;    // vectors per block
constexpr int S2_TK = 32;     // k per chunk of the off-block product
constexpr int S2_NST = 2;     // chunk buffers (loads run one chunk ahead)
constexpr int S2_TLD = 130;   // row stride (doubles) of the right-hand side in LDS

constexpr int S1_LROWS = 64;      // eligible rows whose candidate columns stay in LDS
constexpr int S1_HLD = QMAX + 2;   // row length of the in-batch history (16-byte aligned rows)
constexpr int S1_BLOCK = QMAX * (QMAX + 1) + QMAX * S1_HLD;
constexpr int S1_UNION = (4 * S1K::kWaveDoubles > S1_BLOCK) ? 4 * S1K::kWaveDoubles : S1_BLOCK;

__device__ __forceinline__ bool eligible(double d, double tau, double floor_tol)
{
    return d >= tau && !(tau <= 0.0 && d <= floor_tol);
}

__device__ __forceinline__ void stamp(const Step1Params &P, int g, int64_t batch, int what)
{
    if (P.timeline && batch < P.timeline_cap && g == 0 && threadIdx.x == 0)
        P.timeline[batch * 8 + what] = (int64_t)wall_clock64();
}

// In-batch value of step t: (c - sum_{tp<t} own[tp] piv[tp]) / sqrt(pivot), the
// sum taken in four interleaved partial sums a[tp mod 4], each in increasing
// tp, combined as (a0 + a1) + (a2 + a3).  The row update repeats exactly this
// arithmetic, so candidate rows agree bit for bit with the block
// factorisation.  The steps run in groups of 8 (the step within the group is
// a compile-time index): earlier full groups are read with 16-byte loads and
// the current group's first entries at fixed offsets, so nothing is masked.
__device__ __forceinline__ void inbatch_group(const double *__restrict__ own,
                                              const double *__restrict__ piv, double (&a)[4])
{
    double x[8], y[8];
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
        const double2 xo = *reinterpret_cast<const double2 *>(own + u);
        const double2 yo = *reinterpret_cast<const double2 *>(piv + u);
        x[u] = xo.x;
        x[u + 1] = xo.y;
        y[u] = yo.x;
        y[u + 1] = yo.y;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u & 3] = fma(-x[u], y[u], a[u & 3]);
}

__global__ __launch_bounds__(256) void k_step1(const Step1Batch B)
{
    __shared__ double sU[S1_UNION];   // phase-dependent: nominations / GEMM staging / candidate block
    __shared__ double sD[SMAX];       // residual diagonal of this workgroup's active rows
    __shared__ int sList[SMAX];       // this workgroup's eligible rows (local indices)
    __shared__ int sCand[SMAX];       // local row -> candidate index, or -1
    __shared__ double sC[S1_LROWS][QMAX + 1];   // candidate columns of the first eligible rows
    __shared__ int sQ[QMAX];          // candidate slots
    __shared__ double sQd[QMAX];      // candidate residual diagonals
    __shared__ RowRec sRow[SMAX];     // pair data of this workgroup's active rows
    __shared__ RowRec sQrow[QMAX];    // candidate pair data
    __shared__ int sPiv[QMAX];        // candidate index of in-batch pivot t
    __shared__ double sDp[QMAX];      // pivot values
    __shared__ double sRs[QMAX];      // 1 / sqrt of pivot values
    __shared__ int s_nq, s_kb, s_stop, s_status, s_cnt, s_ns;
    __shared__ int s_prog, s_kbfin, s_lost;   // in-batch pivots published / final count / wait lost
    __shared__ double s_U;
    __shared__ int s_iU;

    Nom *sNom = reinterpret_cast<Nom *>(sU);
    double (*sS)[QMAX + 1] = reinterpret_cast<double (*)[QMAX + 1]>(sU);
    // sH[c][t]: in-batch value of candidate c at in-batch step t
    double (*sH)[S1_HLD] = reinterpret_cast<double (*)[S1_HLD]>(sU + QMAX * (QMAX + 1));

    const int tid = threadIdx.x;
    int mol = 0;
    while (mol + 1 < B.count && (int)blockIdx.x >= B.block_begin[mol + 1]) ++mol;
    const Step1Params &P = B.p[mol];
    const int G = B.block_begin[mol + 1] - B.block_begin[mol];
    const int g = (int)blockIdx.x - B.block_begin[mol];
    const int64_t n_act = P.n_act;
    const int64_t ldT = P.ldT;
    // This workgroup's active rows: slots g, g + G, g + 2G, .. (dealt round
    // robin, so every workgroup holds rows from the whole molecule and about
    // as many of them stay eligible as in any other workgroup: the candidate-
    // column product, which all workgroups wait for, is balanced).  Local row
    // i is slot g + i G; slots ascend with i.
    const int ns = (n_act > g) ? (int)min((int64_t)P.slice, (n_act - g + G - 1) / G) : 0;
    auto slot_of = [&](int i) -> int64_t { return (int64_t)g + (int64_t)i * G; };
    const double tau = P.tau;
    const double ftol = (tau <= 0.0)
        ? (double)P.n_rows * 0x1p-53 * __longlong_as_double((long long)*P.d1max_bits) : 0.0;
    const int q = P.q;
    double *LT = P.LT_act;
    unsigned int gen = 0;

    const int64_t k_first = *P.k_start;
    if (k_first < 0) return;   // a resume whose stored state was invalid (status already set)
    if (*P.n_act_dev != n_act || P.n_rows_dev[0] != P.n_rows) {
        if (g == 0 && tid == 0) *P.status = 5;  // CD_ERR_DEVICE: device and host counts differ
        return;
    }
    for (int i = tid; i < ns; i += 256) {
        sD[i] = P.D_act[slot_of(i)];
        sRow[i] = P.rows[P.act_row[slot_of(i)]];
    }
    int64_t K = k_first;
    int64_t batch = 0;
    int status = 0;
    __syncthreads();

    for (;; ++batch) {
        stamp(P, g, batch, 0);
        // ---- this workgroup's eligible rows (compacted list)
        if (tid < 64) {
            int base = 0;
            for (int c = 0; c < ns; c += 64) {
                int i = c + tid;
                bool e = (i < ns) && eligible(sD[i], tau, ftol);
                unsigned long long mask = __ballot(e);
                unsigned long long below = (tid == 0) ? 0ull : (~0ull >> (64 - tid));
                if (e) sList[base + __popcll(mask & below)] = i;
                base += __popcll(mask);
            }
            if (tid == 0) s_cnt = base;
        }
        // ---- local nominations: the first CNOM+1 own rows in pivot order, picked
        //      by wave 0 (lane l holds rows l, l + 64, ..; a non-finite residual
        //      is nominated as +inf)
        if (tid < 64) {
            double v[4];
            int x[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = tid + 64 * j;
                v[j] = -INFINITY;
                x[j] = 0x7fffffff;
                if (i < ns) {
                    const double d = sD[i];
                    if (d != d || d == INFINITY) {
                        v[j] = INFINITY;
                        x[j] = (int)slot_of(i);
                    } else if (eligible(d, tau, ftol)) {
                        v[j] = d;
                        x[j] = (int)slot_of(i);
                    }
                }
            }
            for (int t = 0; t <= CNOM; ++t) {
                // this lane's first entry (rows ascend with j, so ties keep the lower j)
                int cj = 0;
#pragma unroll
                for (int j = 1; j < 4; ++j) cj = nom_before(v[j], x[j], v[cj], x[cj]) ? j : cj;
                double cd = v[0];
                int cx = x[0];
#pragma unroll
                for (int j = 1; j < 4; ++j) {
                    cd = (cj == j) ? v[j] : cd;
                    cx = (cj == j) ? x[j] : cx;
                }
                const int wl = wave_pick_first(cd, cx);
                Nom e{-INFINITY, 0x7fffffff, 0};
                if (wl >= 0) {
                    e.d = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(cd), wl),
                                           __builtin_amdgcn_readlane(__double2loint(cd), wl));
                    e.idx = __builtin_amdgcn_readlane(cx, wl);
                    if (tid == wl) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) v[j] = (cj == j) ? -INFINITY : v[j];
                    }
                }
                if (tid == 0) sNom[t] = e;
            }
        }
        __syncthreads();
        for (int i = tid; i <= CNOM; i += 256) P.noms[g * (CNOM + 1) + i] = sNom[i];
        if (!grid_barrier(P.gs, G, g, gen, P.spin_limit)) {
            status = 5;
            break;
        }
        stamp(P, g, batch, 1);
        // ---- union of nominations; bound U = first row not nominated anywhere
        //      (the best (CNOM+1)-th nomination over workgroups).  A nomination
        //      that does not come before U can never be accepted in this batch
        //      (its residual only decreases, and the block factorisation stops
        //      at the first pivot that does not come before U), so only the
        //      nominations before U are kept; they are a prefix of the full
        //      union in pivot order, so the candidates and the bound are those
        //      of the full union with the never-accepted rows left out.  With a
        //      span factor eta < 1 every nomination is kept (step 3 may then
        //      accept rows that do not come before U).
        const int nu = G * CNOM;
        Nom mine[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = tid + 256 * r;
            mine[r] = Nom{-INFINITY, 0x7fffffff, 0};
            if (i < nu) mine[r] = P.noms[(i / CNOM) * (CNOM + 1) + (i % CNOM)];
        }
        if (tid < 64) {
            double bd = -INFINITY;
            int bi = 0x7fffffff;
            Nom e[S1_MAXG / 64];   // all loads in flight before the first compare
#pragma unroll
            for (int r = 0; r < S1_MAXG / 64; ++r) {
                const int h = tid + 64 * r;
                e[r] = Nom{-INFINITY, 0x7fffffff, 0};
                if (h < G) e[r] = P.noms[h * (CNOM + 1) + CNOM];
            }
#pragma unroll
            for (int r = 0; r < S1_MAXG / 64; ++r) {
                if (nom_before(e[r].d, e[r].idx, bd, bi)) {
                    bd = e[r].d;
                    bi = e[r].idx;
                }
            }
            int lo;
            wave_best(bd, bi, lo);
            if (tid == 0) {
                s_U = bd;
                s_iU = bi;
                s_ns = 0;
            }
        }
        __syncthreads();
        {
            const double U = s_U;
            const int iU = s_iU;
            const int lane = tid & 63;
            const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
            const bool span = P.eta < 1.0;   // qualified-set acceptance: keep every nomination
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool keep = span ? (mine[r].d != -INFINITY)
                                       : nom_before(mine[r].d, mine[r].idx, U, iU);
                const unsigned long long m = __ballot(keep);
                int base = 0;
                if (lane == 0 && m) base = atomicAdd(&s_ns, __popcll(m));
                base = __shfl(base, 0, 64);
                if (keep) sNom[base + __popcll(m & below)] = mine[r];
            }
        }
        __syncthreads();
        const int n_keep = s_ns;
        int U2 = 32;
        while (U2 < n_keep) U2 <<= 1;
        block_sort_noms(sNom, U2, n_keep);   // entries past n_keep sort as fillers
        if (tid < 64) {   // sorted: the eligible nominations come first
            const unsigned long long ok =
                __ballot(tid < q && tid < U2 && sNom[tid].d != -INFINITY);
            if (tid == 0) s_nq = __popcll(ok);
        }
        if (tid == 0) {
            const int nq = s_nq;
            Nom nxt = (q < U2) ? sNom[q] : Nom{-INFINITY, 0x7fffffff, 0};
            if (nom_before(nxt.d, nxt.idx, s_U, s_iU)) {
                s_U = nxt.d;
                s_iU = nxt.idx;
            }
            s_stop = 0;
            s_status = 0;
            if (nq == 0) s_stop = 1;                          // no eligible row left
            else if (sNom[0].d == INFINITY) { s_stop = 1; s_status = 4; }  // non-finite diagonal
        }
        __syncthreads();
        if (s_stop) {
            status = s_status;
            break;
        }
        const int nq = s_nq;
        // candidates in ascending row order: in the block factorisation the
        // lowest lane among equal residuals is then the lowest row (rule R1)
        if (tid < nq) {
            const int me = sNom[tid].idx;
            int rank = 0;
            for (int j = 0; j < nq; ++j) rank += (sNom[j].idx < me);
            sQ[rank] = me;
            sQd[rank] = sNom[tid].d;     // the residual diagonal as nominated (= D_act)
            sQrow[rank] = P.rows[P.act_row[me]];
        }
        for (int i = tid; i < ns; i += 256) sCand[i] = -1;
        __syncthreads();
        if (tid < nq) {
            const int64_t dq = (int64_t)sQ[tid] - g;
            if (dq >= 0 && dq % G == 0 && dq / G < ns) sCand[dq / G] = tid;
        }
        __syncthreads();
        stamp(P, g, batch, 2);

        // ---- candidate columns on own eligible rows (FP64 MFMA):
        //      C[j][s] = (s|Q_j) - sum_{J<K} L^J_s L^J_{Q_j}
        const int cnt = s_cnt;
        for (int pb = 0; pb < cnt; pb += S1K::kRows) {
            const int rows_m = min(S1K::kRows, cnt - pb);
            const int rt = (rows_m + 15) >> 4;
            f64x4 acc[3][4];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) acc[r][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
            int64_t aoff[S1K::kNA], boff[S1K::kNB];
#pragma unroll
            for (int u = 0; u < S1K::kNA; ++u) {
                const int m = S1K::row_of(u);
                aoff[u] = (m < rows_m) ? slot_of(sList[pb + m]) * ldT : -1;
            }
#pragma unroll
            for (int u = 0; u < S1K::kNB; ++u) {
                const int n = S1K::row_of(u);
                boff[u] = (n < nq) ? (int64_t)sQ[n] * ldT : -1;
            }
            S1K::run(K, rt, LT, aoff, boff, acc, sU);
            // up to 32 rows: the four waves' partial sums side by side, added
            // below in wave order (the same order as the in-place sum)
            constexpr int PR = 32 * 65;
            static_assert(4 * PR <= S1_UNION, "partial sums do not fit");
            if (rt <= 2) S1K::wave_store_partials(acc, rt, sU, PR);
            else S1K::wave_sum_to_lds(acc, rt, sU);
            for (int e = tid; e < rows_m * 64; e += 256) {
                const int m = e >> 6, n = e & 63;
                if (n < nq) {
                    const int li = pb + m;
                    const int64_t slot = slot_of(sList[li]);
                    const int o = m * 65 + n;
                    const double sum =
                        (rt <= 2) ? ((sU[o] + sU[o + PR]) + sU[o + 2 * PR]) + sU[o + 3 * PR] : sU[o];
                    const double v = eri(sRow[sList[li]], sQrow[n]) - sum;
                    if (li < S1_LROWS) sC[li][n] = v;
                    else P.Cbuf[(int64_t)n * n_act + slot] = v;
                    const int ci = sCand[sList[li]];
                    if (ci >= 0) P.Cblk[ci * QMAX + n] = v;   // candidate row: shared block
                }
            }
            __syncthreads();
        }
        stamp(P, g, batch, 3);
        if (!grid_barrier(P.gs, G, g, gen, P.spin_limit)) {
            status = 5;
            break;
        }
        stamp(P, g, batch, 4);

        // ---- in-batch factorisation of the candidate block (every workgroup)
        {
            // the whole [QMAX][QMAX] block in 16-byte loads, all issued before
            // the first use (rows and columns past nq are read, not kept)
            constexpr int NV = QMAX * QMAX / (2 * 256);
            const double2 *src = reinterpret_cast<const double2 *>(P.Cblk);
            double2 v[NV];
#pragma unroll
            for (int u = 0; u < NV; ++u) v[u] = src[tid + 256 * u];
#pragma unroll
            for (int u = 0; u < NV; ++u) {
                const int e = 2 * (tid + 256 * u), i = e / QMAX, j = e % QMAX;
                if (i < nq && j < nq) sS[i][j] = v[u].x;
                if (i < nq && j + 1 < nq) sS[i][j + 1] = v[u].y;
            }
        }
        if (tid == 0) {
            s_prog = 0;
            s_kbfin = -1;
            s_lost = 0;
        }
        __syncthreads();
        // Wave 0 factors the candidate block and publishes every accepted pivot
        // (candidate, value, 1/sqrt, its in-batch values) as soon as it is
        // formed; waves 1-3 apply the pivots to this workgroup's eligible rows
        // one step behind, with the same arithmetic, so candidate rows agree
        // bit for bit.
        if (tid < 64) {
            const int i = tid;
            const bool valid = i < nq;
            double dq = valid ? sQd[i] : -INFINITY;
            const int myslot = valid ? sQ[i] : 0x7fffffff;
            bool used = !valid;
            const double U = s_U;
            const int iU = s_iU;
            const int64_t room = P.max_vectors - K;
            int kb = 0, stop = 0, st = 0;
            bool done = false;
            const double eta = P.eta;
            double dmax0 = 0.0;   // the batch's first pivot: the global maximum residual
            for (int c = 0; c < QMAX / 8 && !done; ++c) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int t = 8 * c + u;
                    const double val = used ? -INFINITY : dq;
                    double bd;
                    const int bl = wave_argmax_pos(val, bd);     // lowest lane = lowest row
                    if (bl < 0) {                                // no positive residual left
                        done = true;
                        break;
                    }
                    const int bi = __builtin_amdgcn_readlane(myslot, bl);
                    dmax0 = (t == 0) ? bd : dmax0;
                    // provably the global argmax, or (span factor < 1) qualified:
                    // residual >= eta times the batch's first pivot
                    const bool first = nom_before(bd, bi, U, iU);
                    const bool qualified = first || (eta < 1.0 && bd >= eta * dmax0);
                    const bool elig = eligible(bd, tau, ftol);      // D >= tau
                    if (!qualified || !elig || t >= room) {
                        // the decomposition ends when the global maximum is below tau,
                        // or when a pivot it needs finds no room (capacity); a qualified
                        // candidate below tau that is not the global maximum only ends
                        // the batch
                        if (first || (qualified && elig)) {
                            stop = 1;
                            st = elig ? 3 : 0;                   // capacity, or done
                        }
                        done = true;
                        break;
                    }
                    const double *pv = sH[bl];
                    double a[4] = {sS[i][bl], 0.0, 0.0, 0.0};
                    for (int cp = 0; cp < c; ++cp) inbatch_group(sH[i] + 8 * cp, pv + 8 * cp, a);
                    const double *ow = sH[i] + 8 * c;
#pragma unroll
                    for (int up = 0; up < u; ++up)
                        a[up & 3] = fma(-ow[up], pv[8 * c + up], a[up & 3]);
                    const double inv = rsqrt_nr(bd);
                    const double lt = ((a[0] + a[1]) + (a[2] + a[3])) * inv;
                    dq = (i == bl) ? 0.0 : fma(-lt, lt, dq);
                    used = used || (i == bl);
                    sH[i][t] = lt;
                    if (i == 0) {
                        sPiv[t] = bl;
                        sDp[t] = bd;
                        sRs[t] = inv;
                    }
                    // LDS operations of one wave are performed in issue order, so a
                    // wave that reads the new count also reads the pivot data
                    // written before it (no wait for the writes is needed here);
                    // the compiler barrier keeps the program order
                    __asm__ volatile("" ::: "memory");
                    if (i == 0)
                        __hip_atomic_store(&s_prog, t + 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    kb = t + 1;
                }
            }
            // a candidate residual that turned NaN inside the batch ends the
            // decomposition (lanes without a candidate carry no value)
            if (__ballot(!used && dq != dq)) {
                stop = 1;
                st = 4;
            }
            if (i == 0) {
                s_kb = kb;
                s_stop = stop;
                s_status = st;
                __hip_atomic_store(&s_kbfin, kb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        } else {
            // ---- apply the accepted pivots to own eligible rows as they appear
            for (int li = tid - 64; li < cnt; li += 192) {
                const int sl = sList[li];
                const int64_t slot = slot_of(sl);
                double d = sD[sl];
                double l[QMAX];
                bool fin = false;
#pragma unroll
                for (int t = 0; t < QMAX; ++t) {
                    if (!fin) {
                        // step t published, or the factorisation ended before it
                        // (bounded: wave 0 always publishes the final count)
                        const uint64_t t0 = wall_clock64();
                        for (;;) {
                            if (__hip_atomic_load(&s_prog, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP) > t)
                                break;
                            const int kf = __hip_atomic_load(&s_kbfin, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP);
                            if (kf >= 0 && kf <= t) {
                                fin = true;
                                break;
                            }
                            if (wall_clock64() - t0 > 100000000ull) {   // 1 s
                                s_lost = 1;
                                fin = true;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                        // the pivot data are read after the count (program order)
                        __asm__ volatile("" ::: "memory");
                    }
                    if (!fin) {
                        const int it = sPiv[t];
                        const double c = (li < S1_LROWS) ? sC[li][it]
                                                         : P.Cbuf[(int64_t)it * n_act + slot];
                        double a[4] = {c, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int tp = 0; tp < t; ++tp) a[tp & 3] = fma(-l[tp], sH[it][tp], a[tp & 3]);
                        l[t] = ((a[0] + a[1]) + (a[2] + a[3])) * sRs[t];
                        d = fma(-l[t], l[t], d);
                        if (sQ[it] == slot) d = 0.0;
                        LT[slot * ldT + K + t] = l[t];
                    }
                }
                sD[sl] = d;
                P.D_act[slot] = d;
            }
        }
        __syncthreads();
        stamp(P, g, batch, 5);
        const int kb = s_kb;
        if (s_lost) {   // a row-update wait ran out of time: CD_ERR_DEVICE
            status = 5;
            break;
        }
        if (g == 0) {
            for (int t = tid; t < kb; t += 256) {
                int slot = sQ[sPiv[t]];
                int row = P.act_row[slot];
                P.pivots[K + t] = row;
                P.piv_slot[K + t] = slot;
                P.dpiv[K + t] = sDp[t];
                if (P.pivot_values) P.pivot_values[K + t] = sDp[t];
                P.pivot_of_row[row] = (int32_t)(K + t);
            }
        }
        K += kb;
        __syncthreads();
        stamp(P, g, batch, 6);
        if (s_stop) {
            status = s_status;
            break;
        }
    }
    if (g == 0 && tid == 0) {
        *P.n_vectors = K;
        *P.status = status;
        if (P.timeline_count) *P.timeline_count = batch + 1;
    }
    if (status == 5 && tid == 0) *P.status = 5;
}

// ---------------------------------------------------------------- pivot block
// Lp[K][J] = L^J at pivot row P_K (J < K), copied from the active-row
// vectors; prow[K] = pair data of pivot row K.  One workgroup per K.
__device__ __forceinline__ int pivot_mol(const int32_t *begin, int count)
{
    int mol = 0;
    while (mol + 1 < count && (int)blockIdx.x >= begin[mol + 1]) ++mol;
    return mol;
}

__global__ __launch_bounds__(256) void k_gather_pivots(const PivotBatch B)
{
    const int mol = pivot_mol(B.gather_begin, B.count);
    const PivotMol &Q = B.m[mol];
    const int64_t M = *Q.n_vectors;
    const int64_t Kc = (int64_t)blockIdx.x - B.gather_begin[mol];
    const int64_t k0 = *Q.k_start;
    if (Kc >= M || k0 < 0 || Kc < k0) return;
    const double *src = Q.LT + (int64_t)Q.piv_slot[Kc] * Q.ldT;
    for (int64_t J = threadIdx.x; J < Kc; J += 256) Q.Lp[Kc * Q.ldp + J] = src[J];
    if (threadIdx.x == 0) Q.prow[Kc] = Q.rows[Q.pivots[Kc]];
}

// Inverse-transposed pivot blocks.  Blocks start at the first vector this
// call forms (k_start: 0, or M1 when resuming).  For the 64 vectors K = b0 + j
// of one block let S be the lower-triangular 64 x 64 matrix S[j][i] = L^{b0+i} at
// pivot row P_{b0+j} (i < j) and S[j][j] = sqrt(d_{b0+j}) (the divisor of the
// vector equation of Sec. 2).  Then the block of vectors obeys T = L_blk S^T,
// T being the right-hand side (r|P_K) - sum over earlier blocks, so
// L_blk = T G with G = S^{-T} (upper triangular).  Lane c solves S x = e_c by
// forward substitution with x in registers (both loops unrolled, four partial
// sums per row, the diagonal applied as a precomputed reciprocal); x is row c
// of G.  In a ragged last block the unused part of S is the identity.  One
// launch covers the blocks of every problem of a pivot-selection launch.
__global__ __launch_bounds__(64) void k_block_inverse(const PivotBatch B)
{
    const int mol = pivot_mol(B.inverse_begin, B.count);
    const PivotMol &Q = B.m[mol];
    const int64_t blk = (int64_t)blockIdx.x - B.inverse_begin[mol];
    const double *__restrict__ Lp = Q.Lp;
    const int64_t ldp = Q.ldp;
    const int64_t k0 = *Q.k_start;
    const int64_t b0 = k0 + blk * 64;
    const int64_t M = *Q.n_vectors;
    if (k0 < 0 || b0 >= M) return;
    const int nb = (int)min((int64_t)64, M - b0);
    __shared__ double sS[64][66];
    __shared__ double sR[64];   // 1 / S[j][j], so the substitution chain holds no division
    const int c = threadIdx.x;
    for (int j = 0; j < 64; ++j) {
        double v = 0.0;
        if (c < j) {
            if (j < nb) v = Lp[(b0 + j) * ldp + b0 + c];
        } else if (c == j) {
            v = (j < nb) ? sqrt(Q.dpiv[b0 + j]) : 1.0;
        }
        sS[j][c] = v;
    }
    __syncthreads();
    sR[c] = 1.0 / sS[c][c];
    __syncthreads();
    double x[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        double a[4] = {(j == c) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < j; ++i) a[i & 3] = fma(-sS[j][i], x[i], a[i & 3]);
        x[j] = ((a[0] + a[1]) + (a[2] + a[3])) * sR[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 64; ++j) sS[c][j] = x[j];
    __syncthreads();
    double *g = Q.G + blk * 4096;
    for (int r = 0; r < 64; ++r) g[r * 64 + c] = sS[r][c];
}

// Inverse-transposed 128 x 128 pivot blocks of the all-row solve, composed from
// the two 64-blocks it holds.  With the pivot block of vectors [b0, b0 + 128)
// split as S = [[S1, 0], [C, S2]] (S1, S2 the 64-blocks of k_block_inverse,
// C[i][j] = L^{b0+j} at pivot row P_{b0+64+i}),
//     S^{-T} = [[G1, X], [0, G2]],  G1 = S1^{-T}, G2 = S2^{-T}, X = -G1 C^T G2.
// The result is written in the operand order of the solve's FP64 MFMA so that
// each lane reads its values as consecutive 16-byte pieces:
//     Gf[blk][cg][s2][lane][e] = G[4 s + lane / 16][16 cg + lane % 16],  s = 2 s2 + e,
// for the 8 column groups cg of 16 columns and the 32 k-steps s of 4.  In a
// ragged last block the unused part of G is the identity (S2 of a ragged block
// is, and C is zero on the missing rows), which the solve never reads into
// a stored vector.
__global__ __launch_bounds__(256) void k_block_g128(const PivotBatch B)
{
    const int mol = pivot_mol(B.g128_begin, B.count);
    const PivotMol &Q = B.m[mol];
    const int64_t blk = (int64_t)blockIdx.x - B.g128_begin[mol];
    const int64_t k0 = *Q.k_start;
    const int64_t b0 = k0 + blk * S2_NB;
    const int64_t M = *Q.n_vectors;
    if (k0 < 0 || b0 >= M) return;
    const int nb2 = (int)min((int64_t)S2_NB, M - b0) - 64;   // vectors of the second half
    __shared__ double sG1[64][65], sG2[64][65], sW[64][65];
    const int tid = threadIdx.x;
    const double *g1 = Q.G + (2 * blk) * 4096, *g2 = g1 + 4096;
    for (int e = tid; e < 4096; e += 256) {
        const int i = e >> 6, j = e & 63;
        sG1[i][j] = g1[e];
        sG2[i][j] = (nb2 > 0) ? g2[e] : 0.0;
        sW[i][j] = (i < nb2) ? Q.Lp[(b0 + 64 + i) * Q.ldp + b0 + j] : 0.0;   // C
    }
    __syncthreads();
    // thread: row i = tid / 4 of a 64 x 64 product, columns 16 (tid % 4) ..
    const int i = tid >> 2, c0 = 16 * (tid & 3);
    double y[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) y[c] = 0.0;
    for (int k = 0; k < 64; ++k) {   // Y = C^T G2
        const double a = sW[k][i];
#pragma unroll
        for (int c = 0; c < 16; ++c) y[c] = fma(a, sG2[k][c0 + c], y[c]);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) sW[i][c0 + c] = y[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) y[c] = 0.0;
    for (int k = 0; k < 64; ++k) {   // X = -G1 Y
        const double a = sG1[i][k];
#pragma unroll
        for (int c = 0; c < 16; ++c) y[c] = fma(a, sW[k][c0 + c], y[c]);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) sW[i][c0 + c] = -y[c];
    __syncthreads();
    double *out = Q.Gf + blk * (S2_NB * S2_NB);
    for (int e = tid; e < S2_NB * S2_NB; e += 256) {
        const int lane = (e >> 1) & 63, s = 2 * ((e >> 7) & 15) + (e & 1), cg = e >> 11;
        const int k = 4 * s + (lane >> 4), n = 16 * cg + (lane & 15);
        double v;
        if (k < 64) v = (n < 64) ? sG1[k][n] : sW[k][n - 64];
        else v = (n < 64) ? 0.0 : sG2[k - 64][n - 64];
        out[e] = v;
    }
}

// ---------------------------------------------------------------- step 2
// Every row r: L[K][r] = [ (r|P_K) - sum_{J<K} L[J][r] Lp[K][J] ] / sqrt(d_K)
// (Sec. 3, Eq. CVsLT), blocked over 128 vectors.  A 512-thread workgroup owns
// 16 RT rows; for each block it forms
//   off-block product  P = A B^T,  A[m][k] = L[k][r0 + m], B[n][k] = Lp[b0 + n][k], k < b0
//   right-hand side    T = (r|P_K) - P   (the ERIs read from L, where k_rhs_eri put them)
//   in-block solve     L_blk = T G       (G: inverse-transposed 128 x 128 pivot block)
// and the final residual diagonal (a row is zeroed when it is chosen as pivot).
//
// Wave w owns 16 of the block's 128 columns (group cg: w for w < 4, 11 - w
// otherwise, so the two waves of a SIMD share the triangular in-block work
// equally) and all RT row tiles, one v_mfma_f64_16x16x4f64 accumulator per
// tile.  The off-block product streams S2_TK-wide k-chunks through S2_NST
// LDS buffers, loaded straight from memory into LDS S2_NST - 1 chunks ahead of
// the products (global_load_lds; one barrier per chunk):
//   A part: [k][m], rows of 16 RT doubles, 4-byte pieces (L's rows have any
//           parity, so 16-byte pieces could be misaligned); lane l of piece
//           v of wave w writes half l % 2 of double 32 (8 v + w) + l / 2;
//   B part: [n][S2_TK k] in 16-byte pieces, the piece of k-pair g of row n
//           stored at g ^ b_swz(n), so the 16 rows one half-wave reads fall
//           on 16 different bank groups.
// Rows past the matrix are read as the tile's last row and columns past the
// block as its last pivot row: finite values in accumulator rows and columns
// that are never stored.  The right-hand side and the block result go through
// one LDS array T of rows of S2_TLD doubles, which reuses the chunk buffers.
// The ERIs of the right-hand side, (r|P_K) for every row r and every vector K
// the solve forms, written into L itself (the solve then replaces each with the
// vector element).  A separate pass: inside the solve the ERI's registers and
// constants crowd the off-block product's loop (its LDS reads then stop running
// ahead of the matrix instructions), and there they cost a phase of every block.
// Grid: x over rows (256 per workgroup, the row record kept in registers),
// y strided over the vectors, z the problem.
__global__ __launch_bounds__(256) void k_rhs_eri(const Step2Batch B)
{
    if ((int)blockIdx.z >= B.count) return;
    const Step2Mol &Q = B.m[blockIdx.z];
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t k0 = *Q.k_start, M = *Q.n_vectors;
    if (k0 < 0 || r >= Q.n_rows) return;
    const RowRec row = Q.rows[r];
    for (int64_t K = k0 + blockIdx.y; K < M; K += gridDim.y)
        Q.L[K * Q.n_rows + r] = eri(row, Q.prow[K]);
}

// B rows of a chunk: S2_TK values, kBPairs 16-byte pairs; a wave's 64 pieces
// cover kBRows rows.  The pair index of row n is XORed with b_swz(n), so the
// 16 rows a quarter-wave reads at one k-pair fall on 16 different 16-byte
// bank groups.
constexpr int kBPairs = S2_TK / 2;
constexpr int kBRows = 64 / kBPairs;
__device__ __forceinline__ int b_swz(int n)
{
    return (S2_TK == 16) ? ((n >> 1) & 7) : (n & 15);
}

template <int RT>
struct S2Lds {
    static constexpr int R = 16 * RT;
    static constexpr int kA = R * S2_TK;                 // A part of a chunk (doubles)
    static constexpr int kB = S2_NB * S2_TK;             // B part of a chunk
    static constexpr int kChunk = kA + kB;
    static constexpr int kT = R * S2_TLD;
    static constexpr int kU = (S2_NST * kChunk > kT) ? S2_NST * kChunk : kT;
    static constexpr int kALoads = kA / 32 / 8;          // 4-byte-piece loads per wave (RT S2_TK / 16)
    static constexpr int kBLoads = kB / 128 / 8;         // 16-byte-piece loads per wave (S2_TK / 8)
    static_assert(kALoads * 32 * 8 == kA && kBLoads * 128 * 8 == kB, "whole loads per wave");
    static_assert(S2_NST >= 2 && S2_NST <= 4, "the chunk loop's waits cover 2 to 4 buffers");
};

template <int RT>
__global__ __launch_bounds__(512) void k_step2(const Step2Batch B)
{
    using S = S2Lds<RT>;
    constexpr int R = S::R;
    int mol = 0;
    while (mol + 1 < B.count && (int)blockIdx.x >= B.tile_begin[mol + 1]) ++mol;
    const Step2Mol &Q = B.m[mol];
    const int64_t n_rows = Q.n_rows;
    const double *__restrict__ Lp = Q.Lp;
    const int64_t ldp = Q.ldp;
    double *__restrict__ L = Q.L;
    const int tile = (int)blockIdx.x - B.tile_begin[mol];
    // optional device-clock stamps of the last problem's first tile, per block
    const bool stamping = B.timeline && mol == B.count - 1 && tile == 0 && threadIdx.x == 0;
    auto mark = [&](int64_t blk, int what) {
        if (stamping && blk < B.tl_cap) B.timeline[blk * 8 + what] = (int64_t)wall_clock64();
    };
    __shared__ __align__(16) double sU[S::kU];
    double *sT = sU;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int cg = (w < 4) ? w : 11 - w;
    const int64_t r0 = (int64_t)tile * R;
    const int rows_here = (int)min((int64_t)R, n_rows - r0);
    const int64_t M = *Q.n_vectors;
    const int64_t k0 = *Q.k_start;   // vectors before k0 are kept as they are
    if (k0 < 0) return;
    double Dfin = 0.0;
    int kp = -1;
    if (tid < rows_here) {
        Dfin = Q.resume ? Q.diag[r0 + tid] : Q.rows[r0 + tid].d1;
        kp = Q.pivot_of_row[r0 + tid];
    }
    __syncthreads();
    // byte offsets of this lane's A pieces from L + kc n_rows + r0 (fixed per tile)
    int64_t aoff[S::kALoads];
#pragma unroll
    for (int v = 0; v < S::kALoads; ++v) {
        const int f = 32 * (8 * v + w) + (lane >> 1);
        const int k = f / R, m = min(f % R, rows_here - 1);
        aoff[v] = ((int64_t)k * n_rows + m) * 8 + 4 * (lane & 1);
    }
    // B pieces: row n and stored k-pair of this lane's piece v
    int bn[S::kBLoads], bk[S::kBLoads];
#pragma unroll
    for (int v = 0; v < S::kBLoads; ++v) {
        const int n = kBRows * (8 * v + w) + lane / kBPairs;
        bn[v] = n;
        bk[v] = 2 * ((lane % kBPairs) ^ b_swz(n));
    }
    // LDS index of this lane's B operand at k-step s: column 16 cg + lane % 16,
    // k = 4 s + lane / 16, i.e. k-pair 2 s + lane / 32, element (lane / 16) % 2
    const int nB = 16 * cg + (lane & 15), swB = b_swz(nB);
    auto b_index = [&](int s) -> int {
        return nB * S2_TK + 2 * ((2 * s + (lane >> 5)) ^ swB) + ((lane >> 4) & 1);
    };

    for (int64_t b0 = k0; b0 < M; b0 += S2_NB) {
        const int nb = (int)min((int64_t)S2_NB, M - b0);
        const int64_t blk = (b0 - k0) / S2_NB;
        mark(blk, 0);
        int64_t boff[S::kBLoads];
#pragma unroll
        for (int v = 0; v < S::kBLoads; ++v) boff[v] = ((int64_t)min(bn[v], nb - 1) * ldp + bk[v]) * 8;
        const char *Abase = reinterpret_cast<const char *>(L + r0);
        const char *Bbase = reinterpret_cast<const char *>(Lp + b0 * ldp);

        // chunk c of the off-block product (k in [16 c, 16 c + 16), k < b0) into buffer 'buf'
        auto load_chunk = [&](int64_t c, int buf) __attribute__((always_inline)) {
            double *st = sU + buf * S::kChunk;
            const int64_t kc = c * S2_TK;
            if (kc + S2_TK <= b0) {
                const char *a = Abase + kc * n_rows * 8;
#pragma unroll
                for (int v = 0; v < S::kALoads; ++v)
                    lds_dma4(a + aoff[v], (lds_void *)(st + 32 * (8 * v + w)));
                const char *b = Bbase + kc * 8;
#pragma unroll
                for (int v = 0; v < S::kBLoads; ++v)
                    lds_dma16(b + boff[v], (lds_void *)(st + S::kA + 128 * (8 * v + w)));
            } else {
                // ragged last chunk (only when k_start is not a multiple of 16):
                // through registers, zeros past b0
                for (int e = tid; e < S::kA; e += 512) {
                    const int k = e / R, m = min(e % R, rows_here - 1);
                    st[e] = (kc + k < b0) ? L[(kc + k) * n_rows + r0 + m] : 0.0;
                }
                for (int e = tid; e < S::kB; e += 512) {
                    const int n = e / S2_TK, k = e % S2_TK;
                    const int at = n * S2_TK + 2 * ((k >> 1) ^ b_swz(n)) + (k & 1);
                    st[S::kA + at] =
                        (kc + k < b0) ? Lp[(b0 + min(n, nb - 1)) * ldp + kc + k] : 0.0;
                }
            }
        };
        f64x4 acc[RT];
        zero_acc(acc);
        const int64_t nch = (b0 + S2_TK - 1) / S2_TK;
#pragma unroll
        for (int c = 0; c < S2_NST - 1; ++c)
            if (c < nch) load_chunk(c, c);
        int buf = 0;   // buffer of chunk c (c % S2_NST)
        for (int64_t c = 0; c < nch; ++c) {
            // own pieces of chunk c landed (those of the next S2_NST - 2 chunks
            // may stay in flight), then a barrier: every wave's pieces of chunk c
            // are in, and every wave is done with the buffer that chunk
            // c + S2_NST - 1 refills
            constexpr int L1 = S::kALoads + S::kBLoads;   // this wave's loads per chunk
            if (c + S2_NST - 2 < nch) wait_vmcnt<(S2_NST - 2) * L1>();
            else if (S2_NST > 3 && c + 1 < nch) wait_vmcnt<L1>();
            else wait_vmcnt<0>();
            lds_barrier();
            if (c + S2_NST - 1 < nch) load_chunk(c + S2_NST - 1, (buf == 0) ? S2_NST - 1 : buf - 1);
            const double *st = sU + buf * S::kChunk;
            buf = (buf == S2_NST - 1) ? 0 : buf + 1;
            const double *sA = st, *sB = st + S::kA;
#pragma unroll
            for (int s = 0; s < S2_TK / 4; ++s) {
                const double b = sB[b_index(s)];
                const int kk = 4 * s + (lane >> 4);
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    const double a = sA[kk * R + 16 * r + (lane & 15)];
                    acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[r], 0, 0, 0);
                }
            }
        }
        // this wave's G operands (k-steps s < 4 (cg + 1): G is upper triangular),
        // in flight while the right-hand side is formed
        double2 gr[16];
        {
            const double2 *gs = reinterpret_cast<const double2 *>(Q.Gf + blk * (S2_NB * S2_NB)) +
                                cg * 1024 + lane;
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2)
                gr[s2] = (s2 < 2 * (cg + 1)) ? gs[64 * s2] : double2{0.0, 0.0};
        }
        __syncthreads();   // the chunk buffers become T
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                sT[(16 * r + mfma_row(lane, v)) * S2_TLD + 16 * cg + (lane & 15)] = acc[r][v];
        __syncthreads();
        mark(blk, 1);
        // right-hand side T = (r|P_K) - P, zero outside the tile's rows and the block's
        // vectors (consecutive threads: consecutive rows of one vector)
        for (int e = tid; e < R * S2_NB; e += 512) {
            const int n = e / R, m = e % R;
            double &t = sT[m * S2_TLD + n];
            t = (m < rows_here && n < nb) ? L[(b0 + n) * n_rows + r0 + m] - t : 0.0;
        }
        __syncthreads();
        mark(blk, 2);
        // in-block solve L_blk = T G over the k-steps where this wave's G columns are nonzero
        zero_acc(acc);
#pragma unroll
        for (int s2 = 0; s2 < 16; ++s2) {
            if (s2 < 2 * (cg + 1)) {   // wave-uniform
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int kk = 4 * (2 * s2 + e) + (lane >> 4);
                    const double b = e ? gr[s2].y : gr[s2].x;
#pragma unroll
                    for (int r = 0; r < RT; ++r) {
                        const double a = sT[(16 * r + (lane & 15)) * S2_TLD + kk];
                        acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[r], 0, 0, 0);
                    }
                }
            }
        }
        // every G load has landed (waves with few columns leave some unread):
        // otherwise the compiler guards the registers they target with a full
        // wait inside the next block's chunk loop, which drains its prefetch
        wait_vmcnt<0>();
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                sT[(16 * r + mfma_row(lane, v)) * S2_TLD + 16 * cg + (lane & 15)] = acc[r][v];
        __syncthreads();
        mark(blk, 3);
        if (tid < rows_here) {
            for (int j = 0; j < nb; ++j) {
                const double l = sT[tid * S2_TLD + j];
                Dfin = fma(-l, l, Dfin);
                if (b0 + j == kp) Dfin = 0.0;
            }
        }
        mark(blk, 4);
        for (int e = tid; e < nb * R; e += 512) {
            const int j = e / R, m = e % R;
            if (m < rows_here) L[(b0 + j) * n_rows + r0 + m] = sT[m * S2_TLD + j];
        }
        __syncthreads();
        mark(blk, 5);
    }
    if (tid < rows_here) Q.diag[r0 + tid] = Dfin;
}

__global__ void k_init_decompose(GridSync *gs, int32_t *status, int64_t *n_vectors,
                                 unsigned long long *d1max_bits, int64_t *k_start)
{
    for (int i = threadIdx.x; i < kMaxGridBlocks * 16; i += blockDim.x) gs->arrive[i] = 0u;
    if (threadIdx.x == 0) {
        gs->release = 0u;
        gs->abort = 0u;
        *status = 0;
        *n_vectors = 0;
        *d1max_bits = 0ull;
        *k_start = 0;
    }
}

// ---------------------------------------------------------------- resume
// Continuing a finished decomposition to a smaller tau.  The pivot order of
// Sec. 2 does not depend on tau (tau only ends the loop), so the selection
// goes on from the stored vectors and residuals.  The stored count M1 becomes
// k_start; a stored state that cannot be continued sets CD_ERR_INVALID_ARG
// and k_start = -1, which every later kernel of the call reads as "skip".
__global__ void k_init_resume(GridSync *gs, int32_t *status, const int64_t *n_vectors,
                              unsigned long long *d1max_bits, int64_t *k_start,
                              int64_t max_vectors)
{
    for (int i = threadIdx.x; i < kMaxGridBlocks * 16; i += blockDim.x) gs->arrive[i] = 0u;
    if (threadIdx.x == 0) {
        gs->release = 0u;
        gs->abort = 0u;
        *d1max_bits = 0ull;
        const int32_t st = *status;
        const int64_t m1 = *n_vectors;
        const bool ok = (st == 0 || st == 3) && m1 >= 0 && m1 <= max_vectors;   // CD_OK, CAPACITY
        *k_start = ok ? m1 : -1;
        *status = ok ? 0 : 1;   // CD_ERR_INVALID_ARG
    }
}

// The pivot selection's state from the stored outputs, for every active slot a
// (row act_row[a]): its residual D_act[a] = diag[row], and its vectors
// LT_act[a][J] = L[J][row] for J < M1 (64 slots x 64 vectors per workgroup,
// transposed through LDS).  Rows chosen as pivots carry a zero residual, so
// they are never chosen again.
__global__ __launch_bounds__(256) void k_resume_state(const int32_t *__restrict__ act_row,
                                                      int64_t n_act, const double *__restrict__ L,
                                                      int64_t n_rows, const double *__restrict__ diag,
                                                      const int64_t *__restrict__ k_start,
                                                      double *__restrict__ LT_act, int64_t ldT,
                                                      double *__restrict__ D_act)
{
    __shared__ double t[64][65];
    __shared__ int32_t s_row[64];
    const int64_t a0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
    const int64_t m1 = *k_start;
    if (m1 < 0) return;
    if (threadIdx.x < 64) {
        const int64_t a = a0 + threadIdx.x;
        s_row[threadIdx.x] = (a < n_act) ? act_row[a] : 0;
        if (blockIdx.y == 0 && a < n_act) D_act[a] = diag[act_row[a]];
    }
    __syncthreads();
    if (j0 >= m1) return;
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int e = threadIdx.x + 256 * j, jj = e >> 6, aa = e & 63;
        v[j] = (j0 + jj < m1 && a0 + aa < n_act) ? L[(j0 + jj) * n_rows + s_row[aa]] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int e = threadIdx.x + 256 * j;
        t[e >> 6][e & 63] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int e = threadIdx.x + 256 * j, aa = e >> 6, jj = e & 63;
        if (a0 + aa < n_act && j0 + jj < m1) LT_act[(a0 + aa) * ldT + j0 + jj] = t[jj][aa];
    }
}

// pivot_of_row of the stored pivots (the all-row solve reads it).
__global__ void k_resume_pivots(const int64_t *__restrict__ pivots, const int64_t *__restrict__ k_start,
                                int64_t max_vectors, int32_t *__restrict__ pivot_of_row)
{
    const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m1 = *k_start;
    if (K < m1 && K < max_vectors) pivot_of_row[pivots[K]] = (int32_t)K;
}

// Test-only poison: the first active row's residual becomes NaN.
__global__ void k_poison_diag(double *D_act, int64_t n_act)
{
    if (threadIdx.x == 0 && n_act > 0) D_act[0] = __longlong_as_double(0x7ff8000000000000ll);
}

}  // namespace cdk

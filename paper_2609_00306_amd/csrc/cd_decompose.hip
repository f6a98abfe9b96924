// Kernels of the threshold-truncated, fully pivoted Cholesky decomposition of
// the ERI matrix over composite pair indices (paper Sec. 2; the two-step
// organisation of Sec. 3 with exact pivoting).
//
//   setup   : pair table, diagonal D1 = (r|r), screening, compaction of the
//             rows and of the "active" rows (D1 >= tau: the only possible
//             pivots, since D never increases -- Sec. 3).
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

__device__ __forceinline__ void row_flags(double d1, double mx, double schwarz, double tau,
                                          bool &keep, bool &act)
{
    keep = sqrt(d1 * mx) >= schwarz;
    act = keep && (d1 >= tau);
}

// Per-256-pair block counts of kept and active rows.
__global__ __launch_bounds__(256) void k_count(int64_t npairs, const double *__restrict__ D1all,
                                               const unsigned long long *d1max_bits,
                                               double schwarz, double tau,
                                               int32_t *__restrict__ cnt_rows,
                                               int32_t *__restrict__ cnt_act)
{
    __shared__ int s_c[2][4];
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mx = __longlong_as_double((long long)*d1max_bits);
    bool keep = false, act = false;
    if (k < npairs) row_flags(D1all[k], mx, schwarz, tau, keep, act);
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
    double tau, const int64_t *__restrict__ off_rows, const int64_t *__restrict__ off_act,
    int64_t n_cap, int64_t na_cap, int64_t *__restrict__ row_pair, RowRec *__restrict__ rows, int32_t *__restrict__ act_row,
    double *__restrict__ D_act, int32_t *__restrict__ pivot_of_row)
{
    __shared__ int s_c[2][4];
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mx = __longlong_as_double((long long)*d1max_bits);
    bool keep = false, act = false;
    if (k < npairs) row_flags(D1all[k], mx, schwarz, tau, keep, act);
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
constexpr int CNOM = 16;       // nominations per workgroup
constexpr int SMAX = 256;      // active rows per workgroup
constexpr int NOMSORT = 4096;  // union capacity (workgroups * CNOM)
constexpr int S1_MAXG = NOMSORT / CNOM;

__device__ __forceinline__ bool eligible(double d, double tau, double floor_tol)
{
    return d >= tau && !(tau <= 0.0 && d <= floor_tol);
}

__global__ __launch_bounds__(256) void k_step1(Step1Params P)
{
    __shared__ double sD[SMAX];
    __shared__ Nom sNom[NOMSORT];                 // sort buffer; reused as B staging
    __shared__ double sS[QMAX][QMAX + 1];         // candidate block
    __shared__ double sLq[QMAX][QMAX + 1];        // in-batch vectors on the candidates
    __shared__ int sQ[QMAX];                      // candidate slots
    __shared__ int sPiv[QMAX];                    // candidate index of in-batch pivot t
    __shared__ double sDp[QMAX];                  // pivot values
    __shared__ double sRs[QMAX];                  // sqrt of pivot values
    __shared__ int s_nq, s_kb, s_stop, s_status;
    __shared__ double s_U;
    __shared__ int s_iU;

    const int tid = threadIdx.x;
    const int G = gridDim.x;
    const int g = blockIdx.x;
    const int64_t n_act = P.n_act;
    const int64_t s0 = (int64_t)g * P.slice;
    const int ns = (int)max((int64_t)0, min((int64_t)P.slice, n_act - s0));
    const double tau = P.tau;
    const double ftol = (tau <= 0.0)
        ? (double)P.n_rows * 0x1p-53 * __longlong_as_double((long long)*P.d1max_bits) : 0.0;
    const int q = P.q;
    unsigned int gen = 0;

    if (*P.n_act_dev != n_act) {
        if (g == 0 && tid == 0) *P.status = 5;  // CD_ERR_DEVICE: device and host counts differ
        return;
    }
    for (int i = tid; i < ns; i += 256) sD[i] = P.D_act[s0 + i];
    int64_t K = 0;
    int status = 0;
    __syncthreads();

    for (;;) {
        // ---- local nominations: first CNOM+1 own rows in pivot order
        int P2 = 32;
        while (P2 < ns) P2 <<= 1;
        for (int i = tid; i < P2; i += 256) {
            Nom e;
            e.d = -INFINITY;
            e.idx = 0x7fffffff;
            e.pad = 0;
            if (i < ns) {
                double d = sD[i];
                if (d != d || d == INFINITY) {
                    e.d = INFINITY;
                    e.idx = (int)(s0 + i);
                } else if (eligible(d, tau, ftol)) {
                    e.d = d;
                    e.idx = (int)(s0 + i);
                }
            }
            sNom[i] = e;
        }
        __syncthreads();
        block_sort_noms(sNom, P2);
        for (int i = tid; i <= CNOM; i += 256) P.noms[g * (CNOM + 1) + i] = sNom[i];
        if (!grid_barrier(P.gs, G, gen, P.spin_limit)) {
            status = 5;
            break;
        }
        // ---- union of nominations; bound = first row not nominated anywhere
        const int nu = G * CNOM;
        int U2 = 32;
        while (U2 < nu) U2 <<= 1;
        for (int i = tid; i < U2; i += 256) {
            Nom e;
            if (i < nu) {
                e = P.noms[(i / CNOM) * (CNOM + 1) + (i % CNOM)];
            } else {
                e.d = -INFINITY;
                e.idx = 0x7fffffff;
                e.pad = 0;
            }
            sNom[i] = e;
        }
        if (tid < 64) {
            double bd = -INFINITY;
            int bi = 0x7fffffff;
            for (int h = tid; h < G; h += 64) {
                Nom e = P.noms[h * (CNOM + 1) + CNOM];
                if (nom_before(e.d, e.idx, bd, bi)) {
                    bd = e.d;
                    bi = e.idx;
                }
            }
            int lo;
            wave_best(bd, bi, lo);
            if (tid == 0) {
                s_U = bd;
                s_iU = bi;
            }
        }
        __syncthreads();
        block_sort_noms(sNom, U2);
        if (tid == 0) {
            int nq = 0;
            while (nq < q && nq < U2 && sNom[nq].d != -INFINITY) ++nq;
            Nom nxt = (q < U2) ? sNom[q] : Nom{-INFINITY, 0x7fffffff, 0};
            if (nom_before(nxt.d, nxt.idx, s_U, s_iU)) {
                s_U = nxt.d;
                s_iU = nxt.idx;
            }
            s_nq = nq;
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
        if (tid < nq) sQ[tid] = sNom[tid].idx;
        __syncthreads();

        // ---- candidate columns on own eligible rows:
        //      C[j][s] = (s|Q_j) - sum_{J<K} L_act[J][s] L_act[J][Q_j]
        {
            double *sB = reinterpret_cast<double *>(sNom);   // [64][QMAX]
            const int nout = ns * nq;
            // outputs in chunks of 8 per thread
            for (int ob = 0; ob < nout; ob += 8 * 256) {
                double acc[8];
                int os[8];
                int oj[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    int o = ob + tid + 256 * u;
                    os[u] = (o < nout) ? (o % ns) : -1;
                    oj[u] = (o < nout) ? (o / ns) : 0;
                    acc[u] = 0.0;
                    if (os[u] >= 0 && !eligible(sD[os[u]], tau, ftol)) os[u] = -1;
                }
                for (int64_t J0 = 0; J0 < K; J0 += 64) {
                    int jc = (int)min((int64_t)64, K - J0);
                    for (int e = tid; e < 64 * QMAX; e += 256) {
                        int jj = e / QMAX, c = e % QMAX;
                        sB[e] = (jj < jc && c < nq) ? P.L_act[(J0 + jj) * n_act + sQ[c]] : 0.0;
                    }
                    __syncthreads();
                    const double *Abase = P.L_act + J0 * n_act + s0;
                    for (int jj = 0; jj < jc; ++jj) {
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            if (os[u] >= 0)
                                acc[u] = fma(Abase[jj * n_act + os[u]], sB[jj * QMAX + oj[u]],
                                             acc[u]);
                        }
                    }
                    __syncthreads();
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (os[u] >= 0) {
                        const RowRec ra = P.rows[P.act_row[s0 + os[u]]];
                        const RowRec rb = P.rows[P.act_row[sQ[oj[u]]]];
                        P.Cbuf[(int64_t)oj[u] * n_act + s0 + os[u]] = eri(ra, rb) - acc[u];
                    }
                }
            }
        }
        if (!grid_barrier(P.gs, G, gen, P.spin_limit)) {
            status = 5;
            break;
        }

        // ---- in-batch factorisation of the candidate block (every workgroup)
        for (int e = tid; e < nq * nq; e += 256) {
            int i = e / nq, j = e % nq;
            sS[i][j] = P.Cbuf[(int64_t)j * n_act + sQ[i]];
        }
        __syncthreads();
        if (tid < 64) {
            const int i = tid;
            const bool valid = i < nq;
            double dq = valid ? P.D_act[sQ[i]] : -INFINITY;
            const int idx = valid ? sQ[i] : 0x7fffffff;
            bool used = !valid;
            const double U = s_U;
            const int iU = s_iU;
            int kb = 0, stop = 0, st = 0;
            // lane i's own in-batch values live in sLq[.][i]
            for (int t = 0; t < QMAX; ++t) {
                double bd = used ? -INFINITY : dq;
                int bi = used ? 0x7fffffff : idx;
                int bl;
                wave_best(bd, bi, bl);
                if (bd != bd) { stop = 1; st = 4; break; }
                if (!nom_before(bd, bi, U, iU)) break;           // may not be the global argmax
                if (!eligible(bd, tau, ftol)) { stop = 1; break; }   // max D < tau: done
                if (K + t >= P.max_vectors) { stop = 1; st = 3; break; }
                const double rs = sqrt(bd);
                double a = sS[i][bl];
                for (int tp = 0; tp < t; ++tp) a = fma(-sLq[tp][i], sLq[tp][bl], a);
                const double lt = a / rs;
                dq = fma(-lt, lt, dq);
                if (i == bl) {
                    dq = 0.0;
                    used = true;
                }
                sLq[t][i] = lt;
                if (i == 0) {
                    sPiv[t] = bl;
                    sDp[t] = bd;
                    sRs[t] = rs;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                kb = t + 1;
            }
            if (i == 0) {
                s_kb = kb;
                s_stop = stop;
                s_status = st;
            }
        }
        __syncthreads();
        const int kb = s_kb;

        // ---- apply the accepted pivots to own eligible rows (same arithmetic
        //      as the candidate block, so candidate rows agree bit for bit)
        for (int sl = tid; sl < ns; sl += 256) {
            double d = sD[sl];
            if (!eligible(d, tau, ftol)) continue;
            const int64_t slot = s0 + sl;
            double l[QMAX];
#pragma unroll
            for (int t = 0; t < QMAX; ++t) {
                if (t < kb) {
                    const int it = sPiv[t];
                    double a = P.Cbuf[(int64_t)it * n_act + slot];
#pragma unroll
                    for (int tp = 0; tp < t; ++tp) a = fma(-l[tp], sLq[tp][it], a);
                    l[t] = a / sRs[t];
                    d = fma(-l[t], l[t], d);
                    if (sQ[it] == slot) d = 0.0;
                    P.L_act[(K + t) * n_act + slot] = l[t];
                }
            }
            sD[sl] = d;
            P.D_act[slot] = d;
        }
        if (g == 0) {
            for (int t = tid; t < kb; t += 256) {
                int slot = sQ[sPiv[t]];
                int row = P.act_row[slot];
                P.pivots[K + t] = row;
                P.piv_slot[K + t] = slot;
                P.dpiv[K + t] = sDp[t];
                P.pivot_of_row[row] = (int32_t)(K + t);
            }
        }
        K += kb;
        __syncthreads();
        if (s_stop) {
            status = s_status;
            break;
        }
    }
    if (g == 0 && tid == 0) {
        *P.n_vectors = K;
        *P.status = status;
    }
    if (status == 5 && tid == 0) *P.status = 5;
}

// ---------------------------------------------------------------- pivot block
// Lp[J][K] = L^J at pivot row P_K  (J < K), from the active-row vectors;
// prow[K] = pair data of pivot row K.
__global__ __launch_bounds__(256) void k_gather_pivots(const double *__restrict__ L_act,
                                                       int64_t n_act,
                                                       const int32_t *__restrict__ piv_slot,
                                                       const int64_t *__restrict__ pivots,
                                                       const RowRec *__restrict__ rows,
                                                       const int64_t *__restrict__ n_vectors,
                                                       double *__restrict__ Lp, int64_t ldp,
                                                       RowRec *__restrict__ prow)
{
    const int64_t M = *n_vectors;
    const int64_t J = blockIdx.y;
    if (J >= M) return;
    for (int64_t Kc = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; Kc < M;
         Kc += (int64_t)gridDim.x * blockDim.x) {
        if (Kc > J) Lp[J * ldp + Kc] = L_act[J * n_act + piv_slot[Kc]];
        if (J == 0) prow[Kc] = rows[pivots[Kc]];
    }
}

// ---------------------------------------------------------------- step 2
// Every row r: L[K][r] = [ (r|P_K) - sum_{J<K} L[J][r] Lp[J][K] ] / sqrt(d_K),
// blocked over 64 vectors; the off-block sum is an MFMA tile, the in-block
// part a per-row substitution.  Also the final residual diagonal.
__global__ __launch_bounds__(256) void k_step2(const RowRec *__restrict__ rows, int64_t n_rows,
                                               const RowRec *__restrict__ prow,
                                               const double *__restrict__ dpiv,
                                               const double *__restrict__ Lp, int64_t ldp,
                                               const int32_t *__restrict__ pivot_of_row,
                                               const int64_t *__restrict__ n_vectors,
                                               double *__restrict__ L, double *__restrict__ diag)
{
    __shared__ double sA[TK * TM];
    __shared__ double sB[TK * TN];
    __shared__ double sT[TM][TN + 1];
    __shared__ double sLb[TN][TN + 1];
    __shared__ double sRs[TN];
    __shared__ RowRec sPr[TN];

    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * TM;
    const int64_t M = *n_vectors;
    const int myr = tid;   // rows handled in the substitution (tid < 64)
    double Dfin = 0.0;
    int kp = -1;
    RowRec me;
    if (tid < TM && r0 + myr < n_rows) {
        me = rows[r0 + myr];
        Dfin = me.d1;
        kp = pivot_of_row[r0 + myr];
    }
    for (int64_t b0 = 0; b0 < M; b0 += TN) {
        const int nb = (int)min((int64_t)TN, M - b0);
        TileAcc acc;
        acc.zero();
        mfma_tile_f64(
            0, b0,
            [&](int64_t k, int m) -> double {
                int64_t r = r0 + m;
                return (r < n_rows) ? L[k * n_rows + r] : 0.0;
            },
            [&](int64_t k, int n) -> double {
                return (n < nb) ? Lp[k * ldp + b0 + n] : 0.0;
            },
            acc, sA, sB);
        tile_to_lds(acc, &sT[0][0], TN + 1);
        for (int e = tid; e < TN; e += 256) {
            if (e < nb) {
                sPr[e] = prow[b0 + e];
                sRs[e] = sqrt(dpiv[b0 + e]);
            }
        }
        for (int e = tid; e < TN * TN; e += 256) {
            int jj = e / TN, j = e % TN;
            sLb[jj][j] = (jj < j && j < nb) ? Lp[(b0 + jj) * ldp + b0 + j] : 0.0;
        }
        __syncthreads();
        // right-hand side: (r|P_K) - off-block sum
        for (int e = tid; e < TM * TN; e += 256) {
            int m = e / TN, j = e % TN;
            if (j < nb && r0 + m < n_rows) {
                const RowRec a = rows[r0 + m];
                sT[m][j] = eri(a, sPr[j]) - sT[m][j];
            }
        }
        __syncthreads();
        if (tid < TM && r0 + myr < n_rows) {
            for (int j = 0; j < nb; ++j) {
                double a = sT[myr][j];
                for (int jj = 0; jj < j; ++jj) a = fma(-sT[myr][jj], sLb[jj][j], a);
                double l = a / sRs[j];
                sT[myr][j] = l;
                Dfin = fma(-l, l, Dfin);
                if (b0 + j == kp) Dfin = 0.0;
            }
        }
        __syncthreads();
        for (int e = tid; e < TM * TN; e += 256) {
            int j = e / TM, m = e % TM;
            if (j < nb && r0 + m < n_rows) L[(b0 + j) * n_rows + r0 + m] = sT[m][j];
        }
        __syncthreads();
    }
    if (tid < TM && r0 + myr < n_rows) diag[r0 + myr] = Dfin;
}

__global__ void k_init_decompose(GridSync *gs, int32_t *status, int64_t *n_vectors,
                                 unsigned long long *d1max_bits)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        gs->count = 0;
        gs->gen = 0;
        gs->abort = 0;
        *status = 0;
        *n_vectors = 0;
        *d1max_bits = 0ull;
    }
}

}  // namespace cdk

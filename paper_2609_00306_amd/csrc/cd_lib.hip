// Host side of the C ABI declared in include/cd.h: argument checks, workspace
// layout and stream-ordered launches.  All kernels live in this one
// translation unit (unity build) so that plain hipcc -shared suffices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cd.h"
#include "cd_decompose.hip"
#include "cd_jk.hip"
#include "cd_jk_lp.hip"
#include "cd_mp2.hip"
#include "cd_scf.hip"
#include "cd_zcd.hip"

using namespace cdk;

namespace {

thread_local std::string g_err;

cd_status fail(cd_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

cd_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CD_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return CD_OK;
}

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count)
    {
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += align_up(count * sizeof(T));
        return p;
    }
};

int64_t n_pairs(int64_t N) { return N * (N + 1) / 2; }
int64_t blocks_of(int64_t n, int64_t b) { return (n + b - 1) / b; }

// Workspace layout of one decomposition.
struct DecompWs {
    double *D1all;
    unsigned long long *d1max;
    int32_t *cnt_rows, *cnt_act;
    int64_t *off_rows, *off_act, *totals;
    RowRec *rows;
    int32_t *act_row;
    double *D_act;
    double *LT_act;
    double *Cbuf;
    double *Cblk;
    Nom *noms;
    GridSync *gs;
    int32_t *piv_slot;
    double *dpiv;
    int32_t *pivot_of_row;
    double *Lp;
    RowRec *prow;
    double *Ginv;
    double *Gf;
    int64_t *kstart;
    size_t bytes;
};

// Row stride of the active-row vectors: a multiple of 16 doubles, so every
// row starts on a 128-byte line and 16-byte loads stay aligned.
int64_t ld_act(int64_t mv) { return (mv + 15) / 16 * 16; }

DecompWs carve_decomp(void *ws, int64_t N, int64_t n, int64_t na, int64_t mv)
{
    DecompWs w{};
    Carver c(ws);
    const int64_t np = n_pairs(N);
    const int64_t nblk = std::max<int64_t>(1, blocks_of(np, 256));
    w.D1all = c.take<double>(std::max<int64_t>(1, np));
    w.d1max = c.take<unsigned long long>(1);
    w.cnt_rows = c.take<int32_t>(nblk);
    w.cnt_act = c.take<int32_t>(nblk);
    w.off_rows = c.take<int64_t>(nblk);
    w.off_act = c.take<int64_t>(nblk);
    w.totals = c.take<int64_t>(4);
    w.rows = c.take<RowRec>(std::max<int64_t>(1, n));
    w.act_row = c.take<int32_t>(std::max<int64_t>(1, na));
    w.D_act = c.take<double>(std::max<int64_t>(1, na));
    w.LT_act = c.take<double>(std::max<int64_t>(1, ld_act(mv) * na));
    w.Cbuf = c.take<double>(std::max<int64_t>(1, (int64_t)QMAX * na));
    w.Cblk = c.take<double>((int64_t)QMAX * QMAX);
    w.noms = c.take<Nom>((size_t)S1_MAXG * (CNOM + 1));
    w.gs = c.take<GridSync>(1);
    w.piv_slot = c.take<int32_t>(std::max<int64_t>(1, mv));
    w.dpiv = c.take<double>(std::max<int64_t>(1, mv));
    w.pivot_of_row = c.take<int32_t>(std::max<int64_t>(1, n));
    w.Lp = c.take<double>(std::max<int64_t>(1, mv * ld_act(mv)));
    w.prow = c.take<RowRec>(std::max<int64_t>(1, mv));
    w.Ginv = c.take<double>(std::max<int64_t>(1, blocks_of(mv, 64)) * 64 * 64);
    w.Gf = c.take<double>(std::max<int64_t>(1, blocks_of(mv, S2_NB)) * S2_NB * S2_NB);
    w.kstart = c.take<int64_t>(1);
    w.bytes = c.off;
    return w;
}

struct DevInfo {
    int dev = -1;
    int n_cu = 0;
    int coop_blocks_per_cu = 0;
};

// Compute units and pivot-selection occupancy of the current device, queried
// once per device and kept (every entry point asks for them).
cd_status dev_info(DevInfo &di)
{
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static DevInfo cache[kMaxDev];
    if (hipGetDevice(&di.dev) != hipSuccess) return fail(CD_ERR_DEVICE, "no HIP device");
    if (di.dev >= 0 && di.dev < kMaxDev) {
        std::lock_guard<std::mutex> lock(mu);
        if (cache[di.dev].dev == di.dev) {
            di = cache[di.dev];
            return CD_OK;
        }
    }
    if (hipDeviceGetAttribute(&di.n_cu, hipDeviceAttributeMultiprocessorCount, di.dev) != hipSuccess)
        return fail(CD_ERR_DEVICE, "compute-unit count query failed");
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step1, 256, 0) != hipSuccess)
        return fail(CD_ERR_DEVICE, "occupancy query failed");
    di.coop_blocks_per_cu = nb;
    if (di.dev >= 0 && di.dev < kMaxDev) {
        std::lock_guard<std::mutex> lock(mu);
        cache[di.dev] = di;
    }
    return CD_OK;
}

// Independent problems of one call (the J/K builds, the decomposition setup)
// run on kJkSide internal streams (default priority), forked from and joined
// back to the caller's stream with events, so the short kernels of small
// problems overlap.  A hipGraph capture
// of the caller's stream takes the side streams in as branches.  Created once
// per device; one call at a time enqueues on them (the mutex).  Two side
// streams measured best: with the runtime's four hardware queues per process,
// three or four made the 64-molecule batch slower than none.
constexpr int kJkSide = 2;
struct SideStreams {
    hipStream_t s[kJkSide];
    hipEvent_t fork;
    hipEvent_t join[kJkSide];
    bool ok = false;
};

static std::mutex &side_mutex()
{
    static std::mutex mu;
    return mu;
}

// Called with side_mutex() held.
static cd_status side_streams(int dev, SideStreams *&out);

// Fork of the side streams from the caller's stream, joined back on every
// return path: once fork() has succeeded, the destructor makes 'st' wait for
// everything enqueued on the side streams (also when the call fails half
// way), so work on 'st' after the call is ordered after all of it and a
// graph capture of 'st' is left with no unjoined branch.  Declared after the
// side-stream lock, so it is joined before the lock is released.
class SideFork {
public:
    explicit SideFork(hipStream_t st) : st_(st) {}
    SideFork(const SideFork &) = delete;
    SideFork &operator=(const SideFork &) = delete;
    ~SideFork() { (void)join(); }
    cd_status fork(int dev)
    {
        cd_status s = side_streams(dev, side_);
        if (s) return s;
        if (hipEventRecord(side_->fork, st_) != hipSuccess)
            return fail(CD_ERR_DEVICE, "fork record failed");
        forked_ = true;   // from here on the destructor joins, whatever waits were set up
        for (int k = 0; k < kJkSide; ++k)
            if (hipStreamWaitEvent(side_->s[k], side_->fork, 0) != hipSuccess)
                return fail(CD_ERR_DEVICE, "fork wait failed");
        return CD_OK;
    }
    // Join now; returns the first failure (a failed join leaves 'st' unordered).
    cd_status join()
    {
        if (!forked_) return CD_OK;
        forked_ = false;
        cd_status s = CD_OK;
        for (int k = 0; k < kJkSide; ++k)
            if (hipEventRecord(side_->join[k], side_->s[k]) != hipSuccess ||
                hipStreamWaitEvent(st_, side_->join[k], 0) != hipSuccess)
                if (!s) s = fail(CD_ERR_DEVICE, "join failed");
        return s;
    }
    SideStreams *side() const { return side_; }

private:
    hipStream_t st_;
    SideStreams *side_ = nullptr;
    bool forked_ = false;
};

static cd_status side_streams(int dev, SideStreams *&out)
{
    constexpr int kMaxDev = 64;
    static SideStreams cache[kMaxDev];
    if (dev < 0 || dev >= kMaxDev) return fail(CD_ERR_UNSUPPORTED, "device index %d", dev);
    SideStreams &c = cache[dev];
    if (!c.ok) {
        for (int k = 0; k < kJkSide; ++k)
            if (hipStreamCreateWithFlags(&c.s[k], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&c.join[k], hipEventDisableTiming) != hipSuccess)
                return fail(CD_ERR_DEVICE, "side stream creation failed");
        if (hipEventCreateWithFlags(&c.fork, hipEventDisableTiming) != hipSuccess)
            return fail(CD_ERR_DEVICE, "side event creation failed");
        c.ok = true;
    }
    out = &c;
    return CD_OK;
}


cd_status check_mol(const cd_molecule &m)
{
    if (m.n_basis < 0) return fail(CD_ERR_INVALID_ARG, "n_basis < 0");
    if (m.n_basis > 0 && (!m.xyz || !m.alpha)) return fail(CD_ERR_INVALID_ARG, "null xyz/alpha");
    if ((int64_t)m.n_basis * (m.n_basis + 1) / 2 > (int64_t)INT32_MAX)
        return fail(CD_ERR_UNSUPPORTED, "too many basis functions");
    return CD_OK;
}

cd_status check_opts(const cd_decomp_opts *o)
{
    if (!o) return fail(CD_ERR_INVALID_ARG, "null opts");
    if (!(o->tau >= 0.0) || !(o->schwarz >= 0.0))
        return fail(CD_ERR_INVALID_ARG, "tau and schwarz must be finite and >= 0");
    if (!(o->eta >= 0.0 && o->eta <= 1.0))
        return fail(CD_ERR_INVALID_ARG, "eta must be in [0, 1]");
    if (o->flags & ~(CD_SYNC | CD_RESUME | CD_DEBUG_POISON_DIAG))
        return fail(CD_ERR_INVALID_ARG, "unknown flags 0x%x", o->flags);
    if (o->tuning) {
        const int rt = o->tuning->step2_row_tiles, mr = o->tuning->step1_min_rows;
        const int q = o->tuning->step1_q;
        if (q != 0 && (q < 8 || q > QMAX))
            return fail(CD_ERR_INVALID_ARG, "tuning.step1_q must be 0 or 8..%d", QMAX);
        if (rt != 0 && (rt < 2 || rt > 7))
            return fail(CD_ERR_INVALID_ARG, "tuning.step2_row_tiles must be 0 or 2..7");
        if (mr != 0 && (mr < 16 || mr > SMAX))
            return fail(CD_ERR_INVALID_ARG, "tuning.step1_min_rows must be 0 or 16..%d", SMAX);
    }
    return CD_OK;
}

// Setup kernels: D1 of all pairs, max, counts, prefix sums (+ scatter when
// outputs are given).
cd_status launch_setup(const cd_molecule &m, const cd_decomp_opts *o, const DecompWs &w,
                       int64_t *row_pair, int64_t n_cap, int64_t na_cap, hipStream_t st,
                       bool scatter)
{
    const int64_t np = n_pairs(m.n_basis);
    const int64_t nblk = blocks_of(np, 256);
    if (np == 0) return CD_OK;
    k_diag_all<<<(unsigned)nblk, 256, 0, st>>>(m.n_basis, m.xyz, m.alpha, np, w.D1all, w.d1max);
    k_count<<<(unsigned)nblk, 256, 0, st>>>(np, w.D1all, w.d1max, o->schwarz, o->tau,
                                            m.pivot_fn, w.cnt_rows, w.cnt_act);
    k_scan<<<1, 256, 0, st>>>((int32_t)nblk, w.cnt_rows, w.cnt_act, w.off_rows, w.off_act,
                              w.totals);
    if (scatter)
        k_scatter<<<(unsigned)nblk, 256, 0, st>>>(m.n_basis, m.xyz, m.alpha, np, w.D1all,
                                                  w.d1max, o->schwarz, o->tau, m.pivot_fn,
                                                  w.off_rows,
                                                  w.off_act, n_cap, na_cap, row_pair, w.rows,
                                                  w.act_row, w.D_act, w.pivot_of_row);
    return check_launch("setup kernels");
}

// Built-in tile height of the all-row solve (16 RT rows, RT in 2..7).  One
// workgroup runs per compute unit, so the solve takes ceil(tiles / n_cu) rounds
// of one tile each; a tile of 16 RT rows costs about RT * cost[RT] units
// (taller tiles reuse each pivot-row operand over more rows).  The cheapest RT
// wins, the taller on ties.
int step2_rows_default(const Step2Batch &B, int n_cu)
{
    // per-row cost of one round relative to 64-row tiles, measured on the
    // 1200-function solve (M = 5612)
    static const double cost[8] = {0.0, 0.0, 1.2, 1.04, 1.0, 0.95, 0.92, 0.92};
    int best = 7;
    double best_cost = 0.0;
    for (int rt = 7; rt >= 2; --rt) {
        int64_t tiles = 0;
        for (int i = 0; i < B.count; ++i) tiles += blocks_of(B.m[i].n_rows, 16 * rt);
        const double c = (double)blocks_of(tiles, std::max(1, n_cu)) * rt * cost[rt];
        if (rt == 7 || c < best_cost) {
            best = rt;
            best_cost = c;
        }
    }
    return best;
}

// The all-row solve of a batch of problems: first the right-hand-side
// integrals of every row against the new pivots (k_rhs_eri, written into L),
// then the substitution (k_step2).
cd_status launch_rhs_batch(const Step2Batch &B, hipStream_t st)
{
    int64_t max_rows = 0;
    for (int i = 0; i < B.count; ++i) max_rows = std::max(max_rows, B.m[i].n_rows);
    if (max_rows == 0) return CD_OK;
    k_rhs_eri<<<dim3((unsigned)blocks_of(max_rows, 256), 64, (unsigned)B.count), 256, 0, st>>>(B);
    return check_launch("all-row integrals");
}

cd_status launch_step2_batch(Step2Batch &B, int n_cu, int rt_req, hipStream_t st)
{
    const int rt = rt_req ? rt_req : step2_rows_default(B, n_cu);
    B.tile_begin[0] = 0;
    for (int i = 0; i < B.count; ++i)
        B.tile_begin[i + 1] = B.tile_begin[i] + (int32_t)blocks_of(B.m[i].n_rows, 16 * rt);
    const unsigned grid = (unsigned)B.tile_begin[B.count];
    if (grid == 0) return CD_OK;
#define CD_STEP2(RT)                                 \
    case RT:                                         \
        k_step2<RT><<<grid, 512, 0, st>>>(B);        \
        break;
    switch (rt) {
        CD_STEP2(2)
        CD_STEP2(3)
        CD_STEP2(4)
        CD_STEP2(5)
        CD_STEP2(6)
        CD_STEP2(7)
    }
#undef CD_STEP2
    return check_launch("all-row solve");
}

Step1Params step1_params(const cd_problem &p, const DecompWs &w, const cd_decomp_opts *o,
                         int slice, bool with_timeline)
{
    Step1Params P1{};
    P1.rows = w.rows;
    P1.act_row = w.act_row;
    P1.n_act_dev = w.totals + 1;
    P1.n_act = p.n_active;
    P1.D_act = w.D_act;
    P1.LT_act = w.LT_act;
    P1.ldT = ld_act(p.max_vectors);
    P1.n_rows_dev = w.totals;
    P1.Cbuf = w.Cbuf;
    P1.Cblk = w.Cblk;
    P1.noms = w.noms;
    P1.gs = w.gs;
    P1.pivots = p.pivots;
    P1.piv_slot = w.piv_slot;
    P1.dpiv = w.dpiv;
    P1.pivot_of_row = w.pivot_of_row;
    P1.n_vectors = p.n_vectors;
    P1.status = p.status;
    P1.k_start = w.kstart;
    P1.pivot_values = p.pivot_values;
    P1.tau = o->tau;
    P1.d1max_bits = w.d1max;
    P1.n_rows = p.n_rows;
    P1.max_vectors = p.max_vectors;
    P1.q = (o->tuning && o->tuning->step1_q) ? o->tuning->step1_q : QMAX;
    P1.eta = (o->eta > 0.0 && o->eta < 1.0) ? o->eta : 1.0;
    P1.slice = slice;
    P1.spin_limit = 1u << 22;
    const bool tl = with_timeline && o->timeline;
    P1.timeline = tl ? o->timeline + 1 : nullptr;
    P1.timeline_count = tl ? o->timeline : nullptr;
    P1.timeline_cap = tl ? o->timeline_cap : 0;
    return P1;
}

}  // namespace

extern "C" {

const char *cd_last_error(void) { return g_err.c_str(); }

const char *cd_version(void) { return "cd-mi355x 0.1 (gfx950)"; }

cd_status cd_query(const cd_molecule *mols, int32_t count, const cd_decomp_opts *opts,
                   const int64_t *max_vectors, cd_sizes *sizes, void *stream)
{
    if (count < 0 || (count > 0 && (!mols || !max_vectors || !sizes)))
        return fail(CD_ERR_INVALID_ARG, "null argument");
    cd_status s = check_opts(opts);
    if (s) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int32_t i = 0; i < count; ++i) {
        if ((s = check_mol(mols[i]))) return s;
        if (max_vectors[i] < 0) return fail(CD_ERR_INVALID_ARG, "max_vectors < 0");
        const int64_t N = mols[i].n_basis;
        int64_t tot[2] = {0, 0};
        if (N > 0) {
            DecompWs probe = carve_decomp(nullptr, N, 0, 0, 0);
            void *tmp = nullptr;
            if (hipMalloc(&tmp, probe.bytes) != hipSuccess)
                return fail(CD_ERR_DEVICE, "hipMalloc of %zu bytes failed", probe.bytes);
            DecompWs w = carve_decomp(tmp, N, 0, 0, 0);
            k_init_decompose<<<1, 256, 0, st>>>(w.gs, w.cnt_rows, w.totals, w.d1max, w.kstart);
            s = launch_setup(mols[i], opts, w, nullptr, 0, 0, st, false);
            if (!s && hipMemcpyAsync(tot, w.totals, sizeof tot, hipMemcpyDeviceToHost, st) !=
                          hipSuccess)
                s = fail(CD_ERR_DEVICE, "copy of row counts failed");
            if (!s && hipStreamSynchronize(st) != hipSuccess)
                s = fail(CD_ERR_DEVICE, "stream synchronise failed");
            (void)hipFree(tmp);
            if (s) return s;
        }
        sizes[i].n_rows = tot[0];
        sizes[i].n_active = tot[1];
        sizes[i].ws_bytes = carve_decomp(nullptr, N, tot[0], tot[1], max_vectors[i]).bytes;
    }
    return CD_OK;
}

}  // extern "C"

namespace {

// Host checks of cd_decompose's problems; 'need' receives the workspace bytes.
cd_status check_decompose(const cd_problem *probs, int32_t count, const cd_decomp_opts *opts,
                          size_t &need)
{
    if (count < 0 || (count > 0 && !probs)) return fail(CD_ERR_INVALID_ARG, "null problems");
    cd_status s = check_opts(opts);
    if (s) return s;
    need = 0;
    for (int32_t i = 0; i < count; ++i) {
        const cd_problem &p = probs[i];
        if ((s = check_mol(p.mol))) return s;
        if (p.max_vectors < 0 || p.n_rows < 0 || p.n_active < 0 || p.n_active > p.n_rows)
            return fail(CD_ERR_INVALID_ARG, "problem %d: bad sizes", i);
        if (p.n_rows > n_pairs(p.mol.n_basis))
            return fail(CD_ERR_INVALID_ARG, "problem %d: n_rows exceeds N(N+1)/2", i);
        if (!p.n_vectors || !p.status) return fail(CD_ERR_INVALID_ARG, "null n_vectors/status");
        if (p.n_rows > 0 && (!p.row_pair || !p.diag))
            return fail(CD_ERR_INVALID_ARG, "null row_pair/diag");
        if (p.n_rows > 0 && p.max_vectors > 0 && (!p.L || !p.pivots))
            return fail(CD_ERR_INVALID_ARG, "null L/pivots");
        if (p.max_vectors > 65535) return fail(CD_ERR_UNSUPPORTED, "max_vectors > 65535");
        need += carve_decomp(nullptr, p.mol.n_basis, p.n_rows, p.n_active, p.max_vectors).bytes;
    }
    return CD_OK;
}

// The decomposition of checked problems with the workspace at 'ws' (256-byte
// aligned, large enough).  With 'use_side' and count > 1 the per-problem setup
// runs on the library's side streams; otherwise everything is on 'st'.
cd_status decompose_impl(const cd_problem *probs, int32_t count, const cd_decomp_opts *opts,
                         void *ws, hipStream_t st, bool use_side)
{
    cd_status s = CD_OK;
    DevInfo di;
    if ((s = dev_info(di))) return s;
    // the pivot selection holds at most SMAX active rows per workgroup and one
    // workgroup per compute unit (at most S1_MAXG): refused before any device work
    for (int32_t i = 0; i < count; ++i) {
        const int64_t g_need = blocks_of(probs[i].n_active, SMAX);
        if (probs[i].max_vectors > 0 && g_need > std::min(di.n_cu, S1_MAXG))
            return fail(CD_ERR_UNSUPPORTED,
                        "problem %d: %lld active rows exceed the pivot-selection capacity "
                        "(%d rows per workgroup, %d workgroups)",
                        i, (long long)probs[i].n_active, SMAX, std::min(di.n_cu, S1_MAXG));
    }

    auto record = [&](int k) -> cd_status {
        if (opts->events && hipEventRecord(static_cast<hipEvent_t>(opts->events[k]), st) != hipSuccess)
            return fail(CD_ERR_INVALID_ARG, "timing event %d could not be recorded", k);
        return CD_OK;
    };
    std::vector<DecompWs> W(count);
    {
        char *wbase = static_cast<char *>(ws);
        for (int32_t i = 0; i < count; ++i) {
            const cd_problem &p = probs[i];
            W[i] = carve_decomp(wbase, p.mol.n_basis, p.n_rows, p.n_active, p.max_vectors);
            wbase += W[i].bytes;
        }
    }
    // ---- pair table, diagonal, screening
    if ((s = record(0))) return s;
    const bool resume = (opts->flags & CD_RESUME) != 0;
    {
        // independent problems on the side streams, joined before the selection
        std::unique_lock<std::mutex> side_lock(side_mutex(), std::defer_lock);
        SideFork side(st);
        if (use_side && count > 1) {
            side_lock.lock();
            if ((s = side.fork(di.dev))) return s;
        }
        for (int32_t i = 0; i < count; ++i) {
            const cd_problem &p = probs[i];
            const DecompWs &w = W[i];
            const hipStream_t sp = side.side() ? side.side()->s[i % kJkSide] : st;
            if (resume)
                k_init_resume<<<1, 256, 0, sp>>>(w.gs, p.status, p.n_vectors, w.d1max, w.kstart,
                                                 p.max_vectors);
            else
                k_init_decompose<<<1, 256, 0, sp>>>(w.gs, p.status, p.n_vectors, w.d1max,
                                                    w.kstart);
            if ((s = launch_setup(p.mol, opts, w, p.row_pair, p.n_rows, p.n_active, sp, true)))
                return s;
            if (resume && p.n_active > 0 && p.max_vectors > 0) {
                // the selection's state from the stored vectors and residuals
                k_resume_state<<<dim3((unsigned)blocks_of(p.n_active, 64),
                                      (unsigned)blocks_of(p.max_vectors, 64)),
                                 256, 0, sp>>>(w.act_row, p.n_active, p.L, p.n_rows, p.diag,
                                               w.kstart, w.LT_act, ld_act(p.max_vectors), w.D_act);
                k_resume_pivots<<<(unsigned)blocks_of(p.max_vectors, 256), 256, 0, sp>>>(
                    p.pivots, w.kstart, p.max_vectors, w.pivot_of_row);
            }
            if (opts->flags & CD_DEBUG_POISON_DIAG)
                k_poison_diag<<<1, 64, 0, sp>>>(w.D_act, p.n_active);
            if ((s = check_launch("setup kernels"))) return s;
        }
        if ((s = side.join())) return s;
    }
    if ((s = record(1))) return s;

    // ---- pivot selection: problems share cooperative launches (largest first)
    const int capacity = std::min(di.n_cu * std::max(1, di.coop_blocks_per_cu), kMaxGridBlocks * 64);
    const int gcap = std::min(di.n_cu, S1_MAXG);
    std::vector<int> order;
    for (int32_t i = 0; i < count; ++i)
        if (probs[i].n_active > 0 && probs[i].max_vectors > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return probs[a].n_active > probs[b].n_active; });
    auto gmin = [&](int i) { return (int)blocks_of(probs[i].n_active, SMAX); };
    const int min_rows = (opts->tuning && opts->tuning->step1_min_rows) ? opts->tuning->step1_min_rows
                                                                         : 32;
    auto gmax = [&](int i) {
        int g = (int)std::min<int64_t>(gcap,
                                       std::max<int64_t>(1, blocks_of(probs[i].n_active, min_rows)));
        return std::max(g, gmin(i));
    };
    size_t pos = 0;
    while (pos < order.size()) {
        std::vector<int> grp;
        int sum_min = 0;
        while (pos < order.size() && (int)grp.size() < kStep1Batch &&
               sum_min + gmin(order[pos]) <= capacity) {
            sum_min += gmin(order[pos]);
            grp.push_back(order[pos++]);
        }
        // workgroups per problem: as many as useful, scaled down to fit the GPU
        std::vector<int> G(grp.size());
        int tot = 0;
        for (size_t j = 0; j < grp.size(); ++j) tot += (G[j] = gmax(grp[j]));
        if (tot > capacity) {
            const int64_t want = tot;
            for (size_t j = 0; j < grp.size(); ++j)
                G[j] = std::max(gmin(grp[j]), (int)((int64_t)G[j] * capacity / want));
            tot = 0;
            for (size_t j = 0; j < grp.size(); ++j) tot += G[j];
            while (tot > capacity) {
                size_t big = 0;
                for (size_t j = 0; j < grp.size(); ++j)
                    if (G[j] - gmin(grp[j]) > G[big] - gmin(grp[big])) big = j;
                if (G[big] <= gmin(grp[big])) break;
                --G[big];
                --tot;
            }
        }
        Step1Batch B{};
        B.count = (int32_t)grp.size();
        B.block_begin[0] = 0;
        for (size_t j = 0; j < grp.size(); ++j) {
            const int i = grp[j];
            const int slice = (int)blocks_of(probs[i].n_active, G[j]);
            B.p[j] = step1_params(probs[i], W[i], opts, slice, i == count - 1);
            B.block_begin[j + 1] = B.block_begin[j] + (int32_t)blocks_of(probs[i].n_active, slice);
        }
        void *args[] = {&B};
        const int nblk = B.block_begin[B.count];
        hipError_t e = hipLaunchCooperativeKernel((const void *)k_step1, dim3(nblk), dim3(256),
                                                  args, 0, st);
        if (e != hipSuccess)
            return fail(CD_ERR_DEVICE, "pivot-selection launch (%d workgroups): %s", nblk,
                        hipGetErrorString(e));
        // pivot rows and pivot-block inverses of the whole group, one launch each
        PivotBatch PB{};
        PB.count = (int32_t)grp.size();
        PB.gather_begin[0] = 0;
        PB.inverse_begin[0] = 0;
        PB.g128_begin[0] = 0;
        for (size_t j = 0; j < grp.size(); ++j) {
            const int i = grp[j];
            const cd_problem &p = probs[i];
            PivotMol &q = PB.m[j];
            q.LT = W[i].LT_act;
            q.ldT = ld_act(p.max_vectors);
            q.piv_slot = W[i].piv_slot;
            q.pivots = p.pivots;
            q.rows = W[i].rows;
            q.n_vectors = p.n_vectors;
            q.Lp = W[i].Lp;
            q.ldp = ld_act(p.max_vectors);
            q.prow = W[i].prow;
            q.dpiv = W[i].dpiv;
            q.G = W[i].Ginv;
            q.Gf = W[i].Gf;
            q.k_start = W[i].kstart;
            PB.gather_begin[j + 1] = PB.gather_begin[j] + (int32_t)p.max_vectors;
            PB.inverse_begin[j + 1] = PB.inverse_begin[j] + (int32_t)blocks_of(p.max_vectors, 64);
            PB.g128_begin[j + 1] = PB.g128_begin[j] + (int32_t)blocks_of(p.max_vectors, S2_NB);
        }
        k_gather_pivots<<<(unsigned)PB.gather_begin[PB.count], 256, 0, st>>>(PB);
        k_block_inverse<<<(unsigned)PB.inverse_begin[PB.count], 64, 0, st>>>(PB);
        k_block_g128<<<(unsigned)PB.g128_begin[PB.count], 256, 0, st>>>(PB);
        if ((s = check_launch("pivot gather"))) return s;
    }
    // ---- all-row solve, up to kStep2Batch problems per launch: the integral
    //      passes, then (from event 2 on) the substitutions
    std::vector<Step2Batch> S2;
    for (int32_t i0 = 0; i0 < count; i0 += kStep2Batch) {
        Step2Batch B{};
        for (int32_t i = i0; i < count && B.count < kStep2Batch; ++i) {
            const cd_problem &p = probs[i];
            if (p.n_rows == 0) continue;
            Step2Mol &q = B.m[B.count++];
            q.rows = W[i].rows;
            q.n_rows = p.n_rows;
            q.prow = W[i].prow;
            q.Lp = W[i].Lp;
            q.Gf = W[i].Gf;
            q.ldp = ld_act(p.max_vectors);
            q.pivot_of_row = W[i].pivot_of_row;
            q.n_vectors = p.n_vectors;
            q.L = p.L;
            q.diag = p.diag;
            q.k_start = W[i].kstart;
            q.resume = resume ? 1 : 0;
        }
        const bool last = (i0 + kStep2Batch >= count);
        B.timeline = (last && opts->timeline) ? opts->timeline + 1 + 8 * opts->timeline_cap : nullptr;
        B.tl_cap = opts->timeline ? opts->timeline_cap : 0;
        if (B.count > 0) S2.push_back(B);
    }
    for (const Step2Batch &B : S2)
        if ((s = launch_rhs_batch(B, st))) return s;
    if ((s = record(2))) return s;
    const int rt_req = opts->tuning ? opts->tuning->step2_row_tiles : 0;
    for (Step2Batch &B : S2)
        if ((s = launch_step2_batch(B, di.n_cu, rt_req, st))) return s;
    if ((s = record(3))) return s;

    if (opts->flags & CD_SYNC) {
        if (hipStreamSynchronize(st) != hipSuccess)
            return fail(CD_ERR_DEVICE, "stream synchronise failed");
        for (int32_t i = 0; i < count; ++i) {
            int32_t v = 0;
            if (hipMemcpy(&v, probs[i].status, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
                return fail(CD_ERR_DEVICE, "status copy failed");
            if (v != 0) return fail((cd_status)v, "problem %d: device status %d", i, v);
        }
    }
    return CD_OK;
}

}  // namespace

extern "C" {

cd_status cd_decompose(const cd_problem *probs, int32_t count, const cd_decomp_opts *opts,
                       void *ws, size_t ws_bytes, void *stream)
{
    size_t need = 0;
    cd_status s = check_decompose(probs, count, opts, need);
    if (s) return s;
    if (need > ws_bytes || (need > 0 && !ws))
        return fail(CD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(CD_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    return decompose_impl(probs, count, opts, ws, static_cast<hipStream_t>(stream), true);
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free form
// The workspace of cd_decompose_noalloc: a static device array that every GPU
// the library runs on holds until the process ends.  Host code never uses
// the array's name as an address (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress, once per
// device, with that device current, and is kept per device.
static __device__ __align__(256) unsigned char scratch[CD_NOALLOC_SCRATCH_BYTES];

namespace {

cd_status scratch_address(int dev, void **out)
{
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static void *addr[kMaxDev];
    if (dev < 0 || dev >= kMaxDev) return fail(CD_ERR_UNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CD_ERR_DEVICE, "address of the static scratch: %s", hipGetErrorString(e));
        addr[dev] = p;
    }
    *out = addr[dev];
    return CD_OK;
}

}  // namespace

extern "C" {

cd_status cd_decompose_noalloc(const cd_problem *probs, int32_t count, const cd_decomp_opts *opts,
                               void *stream)
{
    size_t need = 0;
    cd_status s = check_decompose(probs, count, opts, need);
    if (s) return s;
    if (need > (size_t)CD_NOALLOC_SCRATCH_BYTES)
        return fail(CD_ERR_WORKSPACE,
                    "the problems need %zu bytes of workspace; the static scratch holds %zu",
                    need, (size_t)CD_NOALLOC_SCRATCH_BYTES);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(CD_ERR_DEVICE, "no HIP device");
    void *ws = nullptr;
    if ((s = scratch_address(dev, &ws))) return s;
    // every problem on the caller's stream (no side streams)
    return decompose_impl(probs, count, opts, ws, static_cast<hipStream_t>(stream), false);
}

extern "C++" {   // the cache below is C++ (its key is a std::vector)
namespace {
// Shapes measured by cd_autotune in this process, keyed by device and problem shape.
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, cd_tuning> g_tune_cache;

std::vector<int64_t> tune_key(const cd_problem *probs, int32_t count, const cd_decomp_opts *o)
{
    int dev = -1;
    (void)hipGetDevice(&dev);
    auto bits = [](double x) {
        int64_t b;
        std::memcpy(&b, &x, sizeof b);
        return b;
    };
    std::vector<int64_t> k = {dev, count, (int64_t)(o->flags & ~CD_SYNC), bits(o->tau),
                              bits(o->schwarz), bits(o->eta)};
    for (int32_t i = 0; i < count; ++i) {
        const cd_problem &p = probs[i];
        k.insert(k.end(), {p.mol.n_basis, p.n_rows, p.n_active, p.max_vectors,
                           p.mol.pivot_fn ? 1 : 0});
    }
    return k;
}
}  // namespace
}  // extern "C++"

cd_status cd_autotune(const cd_problem *probs, int32_t count, const cd_decomp_opts *opts,
                      void *ws, size_t ws_bytes, cd_tuning *best, void *stream)
{
    if (!best) return fail(CD_ERR_INVALID_ARG, "null best");
    cd_status s = check_opts(opts);
    if (s) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t ev[4] = {};
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &f : ev)
                if (f) (void)hipEventDestroy(f);
            return fail(CD_ERR_DEVICE, "hipEventCreate failed");
        }
    void *evp[4] = {ev[0], ev[1], ev[2], ev[3]};
    cd_tuning t{0, 0, 0};
    cd_decomp_opts o = *opts;
    o.flags = 0;
    o.events = evp;
    o.timeline = nullptr;
    o.timeline_cap = 0;
    o.tuning = &t;
    float sel = 0.f, solve = 0.f;
    // one decomposition with the shape in t; phase times from the events
    auto run = [&]() -> cd_status {
        cd_status r = cd_decompose(probs, count, &o, ws, ws_bytes, stream);
        if (r) return r;
        if (hipStreamSynchronize(st) != hipSuccess)
            return fail(CD_ERR_DEVICE, "stream synchronise failed");
        for (int32_t i = 0; i < count; ++i) {
            int32_t v = 0;
            if (hipMemcpy(&v, probs[i].status, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
                return fail(CD_ERR_DEVICE, "status copy failed");
            if (v != 0) return fail((cd_status)v, "problem %d: device status %d", i, v);
        }
        if (hipEventElapsedTime(&sel, ev[1], ev[2]) != hipSuccess ||
            hipEventElapsedTime(&solve, ev[2], ev[3]) != hipSuccess)
            return fail(CD_ERR_DEVICE, "event timing failed");
        return CD_OK;
    };
    // a shape measured before in this process: one run with the kept result
    const std::vector<int64_t> key = tune_key(probs, count, opts);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            t = it->second;
            s = run();
            for (auto &e : ev) (void)hipEventDestroy(e);
            if (!s) *best = t;
            return s;
        }
    }
    cd_tuning pick{0, 0, 0};
    s = run();   // warm-up with the built-in shapes
    float best_ms = 0.f;
    for (int rt = 2; !s && rt <= 7; ++rt) {
        t = cd_tuning{rt, 0, 0};
        if ((s = run())) break;
        if (rt == 2 || solve < best_ms) {
            best_ms = solve;
            pick.step2_row_tiles = rt;
        }
    }
    const int rows_opts[] = {16, 32, 48, 64};
    for (int k = 0; !s && k < 4; ++k) {
        t = cd_tuning{pick.step2_row_tiles, rows_opts[k], 0};
        if ((s = run())) break;
        if (k == 0 || sel < best_ms) {
            best_ms = sel;
            pick.step1_min_rows = rows_opts[k];
        }
    }
    const int q_opts[] = {32, 48, QMAX};
    for (int k = 0; !s && k < 3; ++k) {
        t = cd_tuning{pick.step2_row_tiles, pick.step1_min_rows, q_opts[k]};
        if ((s = run())) break;
        if (k == 0 || sel < best_ms) {
            best_ms = sel;
            pick.step1_q = q_opts[k];
        }
    }
    if (!s) {
        t = pick;
        s = run();   // leaves the outputs of the chosen shape
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (!s) {
        *best = pick;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = pick;
    }
    return s;
}

// ------------------------------------------------------------------ J / K
namespace {

// k-splits of the exchange product: a multiple of 8 (one XCD per split, see
// syrk_tile_split) giving at least two workgroups per compute unit.
// The FP64 exchange product runs on 128 x 128 tile pairs when their padded
// work is within 1.17x that of 64 x 64 pairs, the speed per issued flop of the
// larger tiles measured on the 1000-function workload (J/K 23.6 -> 20.4 ms,
// both padding N to 1024); 400 functions stay on 64 x 64 tiles (1.13 ms
// against 1.37 ms with 128 x 128).
bool jk_tiles128(int N)
{
    const double t1 = (N + 63) / 64, t2 = (N + 127) / 128;
    return t2 * (t2 + 1) / 2 * 16384.0 < 1.17 * (t1 * (t1 + 1) / 2 * 4096.0);
}

int jk_nsplit(int N, int n_cu)
{
    const int T = (N + 63) / 64;
    const int pairs = T * (T + 1) / 2;
    int ns = (2 * n_cu + pairs - 1) / std::max(1, pairs);
    ns = (ns + 7) / 8 * 8;
    return std::max(8, std::min(ns, 64));
}

// Tile pairs (lower triangle) of the large-tile 3 x BF16 exchange product.
int bx_pairs(int N)
{
    const int T = (N + BX_TILE - 1) / BX_TILE;
    return T * (T + 1) / 2;
}

// k-ranges per XCD of the large-tile 3 x BF16 exchange product: the smallest count whose
// pairs * ss workgroups (one per compute unit) fill the compute units of an
// XCD in whole rounds to 95% or better, else the best fill up to 16.
int bx_subsplits(int pairs, int n_cu)
{
    const double cu_xcd = std::max(1, n_cu / 8);
    int best = 1;
    double best_fill = 0.0;
    for (int ss = 1; ss <= 16; ++ss) {
        const double rounds = pairs * ss / cu_xcd;
        const double fill = rounds / std::ceil(rounds);
        if (fill >= 0.95) return ss;
        if (fill > best_fill + 1e-12) {
            best_fill = fill;
            best = ss;
        }
    }
    return best;
}

// The second half of the transform (k_tr2w): 16-row tiles of a per workgroup
// (even, at most 10: 160 rows), the padded copy of C1 it reads, and the row
// stride of Y / X (whole 128-column tiles).
int tr2_row_tiles(int p) { return std::max(2, std::min(10, 2 * ((p + 31) / 32))); }
int64_t tr2_c1p_ld(int p) { return (int64_t)blocks_of(p, 16 * tr2_row_tiles(p)) * 16 * tr2_row_tiles(p); }
int64_t tr2_c1p_doubles(int64_t N, int p) { return blocks_of(N, TR_TK) * TR_TK * tr2_c1p_ld(p); }
int64_t x_ld(int64_t mv, int64_t q) { return blocks_of(mv * q, 128) * 128; }

// Cp[mu][a] = C[mu][a] (mu < N, a < ncol), zero elsewhere: rows x ld doubles
void launch_pack_c(const double *C, int N, int ncol, int rows, int ld, double *Cp, hipStream_t st)
{
    k_pack_c1<<<(unsigned)std::min<int64_t>(1024, blocks_of((int64_t)rows * ld, 256)), 256, 0, st>>>(
        C, N, ncol, rows, ld, Cp);
}

cd_status launch_tr2(const double *Y, int64_t ldy, int N, const double *C1, int p, int q,
                     const int64_t *n_vectors, int64_t max_vectors, double *C1p, double *Lmo,
                     hipStream_t st)
{
    const int ra = tr2_row_tiles(p);
    const int ldc = (int)tr2_c1p_ld(p);
    const int rows = (int)(blocks_of(N, TR_TK) * TR_TK);
    launch_pack_c(C1, N, p, rows, ldc, C1p, st);
    const dim3 grid((unsigned)blocks_of(max_vectors * (int64_t)q, 128),
                    (unsigned)blocks_of(p, 16 * ra));
    switch (ra) {
    case 2: k_tr2w<2><<<grid, 512, 0, st>>>(Y, ldy, N, C1p, ldc, p, q, n_vectors, Lmo); break;
    case 4: k_tr2w<4><<<grid, 512, 0, st>>>(Y, ldy, N, C1p, ldc, p, q, n_vectors, Lmo); break;
    case 6: k_tr2w<6><<<grid, 512, 0, st>>>(Y, ldy, N, C1p, ldc, p, q, n_vectors, Lmo); break;
    case 8: k_tr2w<8><<<grid, 512, 0, st>>>(Y, ldy, N, C1p, ldc, p, q, n_vectors, Lmo); break;
    default: k_tr2w<10><<<grid, 512, 0, st>>>(Y, ldy, N, C1p, ldc, p, q, n_vectors, Lmo); break;
    }
    return CD_OK;
}

// Number of partial K matrices of the exchange product at a precision.
int jk_splits(int N, int n_cu, cd_precision prec)
{
    if (prec == CD_BF16X3) return 8 * bx_subsplits(bx_pairs(N), n_cu);
    if (prec == CD_FP32) {
        // eight workgroups per compute unit in all (three run at a time): on the
        // 1200-function workload 16 k-ranges took 13.3 ms, 8 took 13.8 ms
        const int T = (N + 63) / 64, pairs = T * (T + 1) / 2;
        int ns = (8 * n_cu + pairs - 1) / std::max(1, pairs);
        ns = (ns + 7) / 8 * 8;
        return std::max(8, std::min(ns, 64));
    }
    if (jk_tiles128(N)) {
        // 128 x 128 pairs, two workgroups per compute unit: the fewest k-ranges
        // (32 to 64, whole per XCD) whose last round of workgroups is at least
        // 80% full (the 1000-function J/K build: 32 k-ranges 20.6 ms, 40 (the
        // choice) 19.8 ms, 48 19.8 ms; 1200 functions: 32 (the choice) and 64
        // 36.7 ms, 48 37.6 ms)
        const int T = (N + 127) / 128, pairs = T * (T + 1) / 2, slots = 2 * std::max(1, n_cu);
        for (int ns = 32; ns < 64; ns += 8) {
            const double r = (double)pairs * ns / slots;
            if (r / std::ceil(r) >= 0.8) return ns;
        }
        return 64;
    }
    return jk_nsplit(N, n_cu);
}

// Unpacking of the packed vectors for the J/K and transform products: a
// dense row map, per-function neighbour lists and the row-major copy LT.
struct SparseWs {
    int32_t *rowof, *deg, *nb_s, *nb_r;
    int64_t *off;
    double *LT;
};

// Row stride of the row-major copy of the vectors: whole 128-vector tiles of
// the half transform, whose 16-byte pieces stay aligned and inside the row.
int64_t lt_ld(int64_t mv) { return blocks_of(mv, HS_P) * HS_P; }

// The padded copy of the coefficients the half transform reads: rows of whole
// column ranges of a workgroup, and one zero row (index N) past the functions.
int64_t hs_cols(int64_t ncol) { return 16 * hs_col_tiles((int)ncol); }
int64_t hs_cp_ld(int64_t ncol) { return blocks_of(ncol, hs_cols(ncol)) * hs_cols(ncol); }

// X^P = Lt^P C over the neighbour lists (k_half_sparse), output form OUT
extern "C++" template <int OUT>
void launch_half(const SparseWs &q, int64_t mv, const double *Cp, int ldcp, int N, int ncol,
                 const int64_t *n_vectors, void *Y, int64_t ldy, int64_t plane, double *Y64,
                 int64_t ldy64, hipStream_t st)
{
    const dim3 grid((unsigned)blocks_of(mv, HS_P), (unsigned)blocks_of(ncol, hs_cols(ncol)),
                    (unsigned)N);
    if (hs_col_tiles(ncol) == 4)
        k_half_sparse<OUT, 4><<<grid, 512, 0, st>>>(q.LT, lt_ld(mv), q.off, q.nb_s, q.nb_r, Cp, ldcp,
                                                   N, ncol, n_vectors, Y, ldy, plane, Y64, ldy64);
    else
        k_half_sparse<OUT, 10><<<grid, 512, 0, st>>>(q.LT, lt_ld(mv), q.off, q.nb_s, q.nb_r, Cp, ldcp,
                                                    N, ncol, n_vectors, Y, ldy, plane, Y64, ldy64);
}
int64_t hs_cp_doubles(int64_t N, int64_t ncol) { return (N + 1) * hs_cp_ld(ncol); }

SparseWs carve_sparse(Carver &c, int64_t N, int64_t n, int64_t mv)
{
    SparseWs w{};
    w.rowof = c.take<int32_t>(std::max<int64_t>(1, N * N));
    w.deg = c.take<int32_t>(std::max<int64_t>(1, N));
    w.off = c.take<int64_t>(N + 1);
    w.nb_s = c.take<int32_t>(std::max<int64_t>(1, 2 * n));
    w.nb_r = c.take<int32_t>(std::max<int64_t>(1, 2 * n));
    w.LT = c.take<double>(std::max<int64_t>(1, n * lt_ld(mv)));
    return w;
}

void launch_sparse_prep(const SparseWs &w, int64_t N, int64_t n, int64_t mv,
                        const int64_t *row_pair, const double *L, const int64_t *n_vectors,
                        hipStream_t st)
{
    const int64_t NN = N * N;
    const unsigned fb = (unsigned)std::min<int64_t>(4096, blocks_of(NN, 256));
    k_fill_i32<<<fb, 256, 0, st>>>(w.rowof, NN, -1);
    k_rowmap<<<(unsigned)blocks_of(n, 256), 256, 0, st>>>(n, row_pair, (int)N, w.rowof);
    k_nbr_count<<<(unsigned)blocks_of(N, 4), 256, 0, st>>>(w.rowof, (int)N, w.deg);
    k_scan_deg<<<1, 256, 0, st>>>(w.deg, (int)N, w.off);
    k_nbr_fill<<<(unsigned)blocks_of(N, 4), 256, 0, st>>>(w.rowof, (int)N, w.off, w.nb_s, w.nb_r);
    k_transpose<<<dim3((unsigned)blocks_of(n, 64), (unsigned)blocks_of(mv, 64)), 256, 0, st>>>(
        L, n, n_vectors, w.LT, lt_ld(mv));
}

struct JkWs {
    double *w, *V, *X, *Kp;
    double *X64;   // FP64 copy of X beside the BF16 planes (3 x BF16 with Lmo)
    double *C1p;   // padded copy of C for the second half of the transform (with Lmo)
    double *Cp;    // padded copy of C for the half transform
    SparseWs sp;
    size_t bytes;
};

// Values per row of a BF16 plane of X (a plane holds bx_rows(N) rows of them,
// k-blocked): a multiple of 8; x_ld's multiple of 128 is also one of XB_K.
int64_t bf16_ld(int64_t n) { return (n + 7) / 8 * 8; }

// Rows of the k-blocked FP32 X and of each BF16 plane: N padded to whole
// 128-row tiles of the exchange product.
int64_t bx_rows(int64_t N) { return (N + BX_TILE - 1) / BX_TILE * BX_TILE; }

JkWs carve_jk(void *ws, const cd_jk_problem &p, int nsplit, cd_precision prec)
{
    JkWs w{};
    Carver c(ws);
    const int64_t N = p.n_basis;
    w.w = c.take<double>(std::max<int64_t>(1, p.n_rows));
    w.V = c.take<double>(std::max<int64_t>(1, p.max_vectors));
    w.sp = carve_sparse(c, N, p.n_rows, p.max_vectors);
    // X: FP64 [N][x_ld(M, O)], or in the same space the k-blocked FP32 X or
    // three k-blocked BF16 planes, each over N rows padded to 128-row tiles
    const int64_t ldx = x_ld(p.max_vectors, p.n_occ);
    const int64_t xf = ldx * N;
    const int64_t xs = (bx_rows(N) * ldx + 1) / 2;
    const int64_t xb = (3 * bx_rows(N) * bf16_ld(ldx) + 3) / 4;
    w.X = c.take<double>(std::max<int64_t>(1, std::max(xf, std::max(xs, xb))));
    w.Kp = c.take<double>(std::max<int64_t>(1, (int64_t)nsplit * N * N));
    w.X64 = (p.Lmo && prec != CD_FP64) ? c.take<double>(std::max<int64_t>(1, xf)) : nullptr;
    w.C1p = p.Lmo ? c.take<double>(std::max<int64_t>(1, tr2_c1p_doubles(N, p.n_occ))) : nullptr;
    w.Cp = c.take<double>(std::max<int64_t>(1, hs_cp_doubles(N, p.n_occ)));
    w.bytes = c.off;
    return w;
}

cd_status check_jk(const cd_jk_problem &p)
{
    if (p.n_basis < 0 || p.n_rows < 0 || p.max_vectors < 0 || p.n_occ < 0)
        return fail(CD_ERR_INVALID_ARG, "negative size");
    if (p.max_vectors > 65535) return fail(CD_ERR_UNSUPPORTED, "max_vectors > 65535");
    if (p.n_basis > 0 && (!p.J || !p.K)) return fail(CD_ERR_INVALID_ARG, "null J/K");
    if (!p.n_vectors || !p.status) return fail(CD_ERR_INVALID_ARG, "null n_vectors/status");
    if (p.n_rows > 0 && (!p.row_pair || (p.max_vectors > 0 && !p.L)))
        return fail(CD_ERR_INVALID_ARG, "null row_pair/L");
    if (p.n_occ > 0 && p.n_basis > 0 && !p.C) return fail(CD_ERR_INVALID_ARG, "null C");
    return CD_OK;
}

}  // namespace

cd_status cd_query_jk(const cd_jk_problem *probs, int32_t count, cd_precision prec,
                      size_t *ws_bytes)
{
    if (count < 0 || (count > 0 && !probs) || !ws_bytes)
        return fail(CD_ERR_INVALID_ARG, "null argument");
    if (prec != CD_FP64 && prec != CD_FP32 && prec != CD_BF16X3)
        return fail(CD_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
    DevInfo di;
    cd_status s = dev_info(di);
    if (s) return s;
    size_t tot = 0;
    for (int32_t i = 0; i < count; ++i) {
        if ((s = check_jk(probs[i]))) return s;
        tot += carve_jk(nullptr, probs[i], jk_splits(probs[i].n_basis, di.n_cu, prec), prec).bytes;
    }
    *ws_bytes = tot;
    return CD_OK;
}

cd_status cd_build_jk(const cd_jk_problem *probs, int32_t count, cd_precision prec,
                      uint32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    size_t need = 0;
    cd_status s = cd_query_jk(probs, count, prec, &need);
    if (s) return s;
    if (need > ws_bytes || (need > 0 && !ws))
        return fail(CD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    DevInfo di;
    if ((s = dev_info(di))) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *wbase = static_cast<char *>(ws);
    std::unique_lock<std::mutex> side_lock(side_mutex(), std::defer_lock);
    SideFork guard(st);
    SideStreams *side = nullptr;
    // several problems: problem i on side stream i mod kJkSide; one problem:
    // its J chain on side stream 0, beside the K chain on the caller's stream
    if (count > 0) {
        side_lock.lock();
        if ((s = guard.fork(di.dev))) return s;
        side = guard.side();
    }
    for (int32_t i = 0; i < count; ++i) {
        const cd_jk_problem &p = probs[i];
        const hipStream_t sp = (count > 1) ? side->s[i % kJkSide] : st;
        const hipStream_t sj = (count > 1) ? sp : side->s[0];   // the J chain
        const int nsplit = jk_splits(p.n_basis, di.n_cu, prec);
        JkWs w = carve_jk(wbase, p, nsplit, prec);
        wbase += w.bytes;
        const int64_t N = p.n_basis, NN = N * N, n = p.n_rows, mv = p.max_vectors;
        const int O = p.n_occ;
        if (N == 0) continue;
        const unsigned fb = (unsigned)std::min<int64_t>(4096, blocks_of(NN, 256));
        k_fill_f64<<<fb, 256, 0, sj>>>(p.J, NN, 0.0);
        k_fill_f64<<<fb, 256, 0, sp>>>(p.K, NN, 0.0);
        if (p.Lmo && n == 0 && O > 0 && mv > 0)
            k_fill_f64<<<256, 256, 0, sp>>>(p.Lmo, mv * O * O, 0.0);
        if (O == 0 || n == 0 || mv == 0) continue;
        launch_sparse_prep(w.sp, N, n, mv, p.row_pair, p.L, p.n_vectors, sp);
        // The order on the problem's stream: the half transform, the second half
        // of the transform (when asked for), the exchange product.  The Coulomb
        // build (the rows' density weights, then two passes over L) runs, for
        // one problem, on side stream 0 beside the exchange product, enqueued
        // after the transform.
        // Measured on the 1200-function workload: the transform beside the
        // exchange product (both bound by the matrix units, and their
        // workgroups mostly cannot share a compute unit) cost 2.7 ms more in FP64
        // and 1.5 ms more in 3 x BF16 than one after the other (FP32: 0.3 ms
        // less); the Coulomb build beside the transpose slowed it from 1.1 to
        // 3 ms (both read L), and beside the half transform it slowed that from
        // 5.7 to 7.4 ms; beside the transform product the J/K build took about
        // 0.3 ms more in FP64 and in 3 x BF16 (0.4 ms less in FP32).
        auto j_chain = [&]() -> cd_status {
            if (sj != sp && (hipEventRecord(side->fork, sp) != hipSuccess ||
                             hipStreamWaitEvent(sj, side->fork, 0) != hipSuccess))
                return fail(CD_ERR_DEVICE, "fork failed");
            k_drow<<<(unsigned)blocks_of(n, 16), 256, 0, sj>>>(n, p.row_pair, O, p.C, w.w);
            k_jV<<<(unsigned)mv, 256, 0, sj>>>(p.L, n, w.w, p.n_vectors, w.V);
            k_jJ<<<(unsigned)blocks_of(n, 64), 256, 0, sj>>>(p.L, n, w.V, p.n_vectors, p.row_pair,
                                                             (int)N, p.J);
            return CD_OK;
        };
        const int ldcp = (int)hs_cp_ld(O);
        launch_pack_c(p.C, (int)N, O, (int)N + 1, ldcp, w.Cp, sp);
        const int T = (int)blocks_of(N, 64);
        const unsigned sgrid = (unsigned)(T * (T + 1) / 2 * nsplit);   // see syrk_tile_split
        const int64_t ldx = x_ld(mv, O);
        float *X32 = reinterpret_cast<float *>(w.X);
        const SparseWs &q = w.sp;
        // the second half of the transform on the FP64 X
        auto second_half = [&](const double *X64) -> cd_status {
            return launch_tr2(X64, ldx, (int)N, p.C, O, O, p.n_vectors, mv, w.C1p, p.Lmo, sp);
        };
        if (prec == CD_FP64) {
            launch_half<HALF_F64>(q, mv, w.Cp, ldcp, (int)N, O, p.n_vectors, w.X, ldx, 0, nullptr, 0,
                                  sp);
            if (p.Lmo && (s = second_half(w.X))) return s;
            if ((s = j_chain())) return s;
            if (jk_tiles128((int)N)) {
                const int T2 = (int)blocks_of(N, 128), pairs2 = T2 * (T2 + 1) / 2;
                k_syrk_rows128<<<(unsigned)(pairs2 * nsplit), 256, 0, sp>>>(w.X, ldx, (int)N, p.n_vectors,
                                                                            O, pairs2, nsplit, w.Kp);
            } else {
                k_syrk_rows<<<sgrid, 256, 0, sp>>>(w.X, ldx, (int)N, p.n_vectors, O, nsplit, w.Kp);
            }
        } else if (prec == CD_FP32) {
            // X in FP64 (matrix cores), written rounded to FP32 (k-blocked; and in
            // FP64 for C^T L C); the exchange product then runs on FP32 matrix cores
            const int64_t R = bx_rows(N);
            launch_half<HALF_F32>(q, mv, w.Cp, ldcp, (int)N, O, p.n_vectors, X32, R, 0, w.X64, ldx,
                                  sp);
            if (p.Lmo && (s = second_half(w.X64))) return s;
            if ((s = j_chain())) return s;
            k_syrk_f32<<<sgrid, 256, 0, sp>>>(X32, R, (int)N, p.n_vectors, O, nsplit, w.Kp);
        } else {
            // X in FP64 (matrix cores), written split into three k-blocked BF16
            // planes; the exchange product then runs on BF16 matrix cores from them
            const int64_t R = bx_rows(N), plane = R * bf16_ld(ldx);
            __bf16 *Xp = reinterpret_cast<__bf16 *>(w.X);
            launch_half<HALF_BF16X3>(q, mv, w.Cp, ldcp, (int)N, O, p.n_vectors, Xp, R, plane, w.X64,
                                     ldx, sp);
            if (p.Lmo && (s = second_half(w.X64))) return s;
            if ((s = j_chain())) return s;
            const int pairs = bx_pairs((int)N);
            k_syrk_bf16x3<<<(unsigned)(pairs * nsplit), 256, 0, sp>>>(
                Xp, R, plane, (int)N, p.n_vectors, O, pairs, nsplit, w.Kp);
        }
        k_kreduce<<<(unsigned)blocks_of(NN, 256), 256, 0, sp>>>(w.Kp, (int)N, nsplit, 0, p.K);
        if ((s = check_launch("J/K kernels"))) return s;
    }
    if ((s = guard.join())) return s;
    if (side_lock.owns_lock()) side_lock.unlock();
    if (flags & CD_SYNC) {
        if (hipStreamSynchronize(st) != hipSuccess)
            return fail(CD_ERR_DEVICE, "stream synchronise failed");
    }
    return CD_OK;
}

// ------------------------------------------------------------------ transform
cd_status cd_query_transform(const cd_transform_problem *probs, int32_t count, size_t *ws_bytes)
{
    if (count < 0 || (count > 0 && !probs) || !ws_bytes)
        return fail(CD_ERR_INVALID_ARG, "null argument");
    size_t tot = 0;
    for (int32_t i = 0; i < count; ++i) {
        const cd_transform_problem &p = probs[i];
        if (p.n_basis < 0 || p.n_rows < 0 || p.max_vectors < 0 || p.p < 0 || p.q < 0)
            return fail(CD_ERR_INVALID_ARG, "negative size");
        if (p.max_vectors > 65535) return fail(CD_ERR_UNSUPPORTED, "max_vectors > 65535");
        Carver c(nullptr);
        carve_sparse(c, p.n_basis, p.n_rows, p.max_vectors);
        c.take<double>(std::max<int64_t>(1, x_ld(p.max_vectors, p.q) * p.n_basis));
        c.take<double>(std::max<int64_t>(1, tr2_c1p_doubles(p.n_basis, p.p)));
        c.take<double>(std::max<int64_t>(1, hs_cp_doubles(p.n_basis, p.q)));
        tot += c.off;
    }
    *ws_bytes = tot;
    return CD_OK;
}

cd_status cd_transform(const cd_transform_problem *probs, int32_t count, uint32_t flags,
                       void *ws, size_t ws_bytes, void *stream)
{
    size_t need = 0;
    cd_status s = cd_query_transform(probs, count, &need);
    if (s) return s;
    if (need > ws_bytes || (need > 0 && !ws))
        return fail(CD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *wbase = static_cast<char *>(ws);
    for (int32_t i = 0; i < count; ++i) {
        const cd_transform_problem &p = probs[i];
        const int64_t N = p.n_basis, n = p.n_rows, mv = p.max_vectors;
        Carver c(wbase);
        SparseWs sp = carve_sparse(c, N, n, mv);
        double *Y = c.take<double>(std::max<int64_t>(1, x_ld(mv, p.q) * N));
        double *C1p = c.take<double>(std::max<int64_t>(1, tr2_c1p_doubles(N, p.p)));
        double *C2p = c.take<double>(std::max<int64_t>(1, hs_cp_doubles(N, p.q)));
        wbase += c.off;
        if (N == 0 || mv == 0 || p.p == 0 || p.q == 0) continue;
        if (!p.Lmo || !p.C1 || !p.C2 || !p.n_vectors || (n > 0 && (!p.L || !p.row_pair)))
            return fail(CD_ERR_INVALID_ARG, "null pointer in transform problem %d", i);
        const int64_t ldy = x_ld(mv, p.q);
        if (n > 0) {
            launch_sparse_prep(sp, N, n, mv, p.row_pair, p.L, p.n_vectors, st);
            const int ldcp = (int)hs_cp_ld(p.q);
            launch_pack_c(p.C2, (int)N, p.q, (int)N + 1, ldcp, C2p, st);
            launch_half<HALF_F64>(sp, mv, C2p, ldcp, (int)N, p.q, p.n_vectors, Y, ldy, 0, nullptr, 0,
                                  st);
        } else {
            k_fill_f64<<<256, 256, 0, st>>>(Y, ldy * N, 0.0);
        }
        launch_tr2(Y, ldy, (int)N, p.C1, p.p, p.q, p.n_vectors, mv, C1p, p.Lmo, st);
        if ((s = check_launch("transform kernels"))) return s;
    }
    if (flags & CD_SYNC) {
        if (hipStreamSynchronize(st) != hipSuccess)
            return fail(CD_ERR_DEVICE, "stream synchronise failed");
    }
    return CD_OK;
}

cd_status cd_one_electron(const cd_one_electron_problem *p, uint32_t flags, void *stream)
{
    if (!p) return fail(CD_ERR_INVALID_ARG, "null problem");
    cd_status s = check_mol(p->mol);
    if (s) return s;
    const int N = p->mol.n_basis;
    if (p->n_charges < 0) return fail(CD_ERR_INVALID_ARG, "n_charges < 0");
    if (p->n_charges > 0 && (!p->charge_xyz || !p->charge))
        return fail(CD_ERR_INVALID_ARG, "null charges");
    if (N > 0 && (!p->S || !p->H)) return fail(CD_ERR_INVALID_ARG, "null S/H");
    if ((int64_t)N * N > ((int64_t)1 << 40)) return fail(CD_ERR_UNSUPPORTED, "basis too large");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n2 = (int64_t)N * N;
    if (n2 > 0)
        k_one_electron<<<(unsigned)blocks_of(n2, 256), 256, 0, st>>>(
            N, p->mol.xyz, p->mol.alpha, p->n_charges, p->charge_xyz, p->charge, p->S, p->H);
    if ((s = check_launch("one-electron kernel"))) return s;
    if ((flags & CD_SYNC) && hipStreamSynchronize(st) != hipSuccess)
        return fail(CD_ERR_DEVICE, "stream synchronise failed");
    return CD_OK;
}

// Device workspace of cd_scf: eight N x N matrices, the Cholesky scratch, the
// reduction results, and the J/K workspace.
struct ScfWs {
    double *X, *A, *B, *T, *W1, *W2, *J, *K, *dres, *red, *Fh, *Eh, *part, *gpart;
    void *jk;
    size_t jk_bytes;
};

static cd_jk_problem scf_jk_problem(const cd_scf_problem &p, double *J, double *K)
{
    cd_jk_problem q{};
    q.n_basis = p.n_basis;
    q.n_rows = p.n_rows;
    q.max_vectors = p.max_vectors;
    q.row_pair = p.row_pair;
    q.L = p.L;
    q.n_vectors = p.n_vectors;
    q.n_occ = p.n_occ;
    q.C = p.C;
    q.J = J;
    q.K = K;
    q.status = p.status;
    return q;
}

static cd_status scf_carve(const cd_scf_problem &p, cd_precision prec, void *base, ScfWs &w,
                           size_t &bytes)
{
    const int64_t n2 = std::max<int64_t>(1, (int64_t)p.n_basis * p.n_basis);
    Carver c(base);
    w.X = c.take<double>(n2);
    w.A = c.take<double>(n2);
    w.B = c.take<double>(n2);
    w.T = c.take<double>(n2);
    w.W1 = c.take<double>(n2);
    w.W2 = c.take<double>(n2);
    w.J = c.take<double>(n2);
    w.K = c.take<double>(n2);
    w.dres = c.take<double>(std::max(1, p.n_basis));
    w.red = c.take<double>(8);
    w.part = c.take<double>(SCF_DIIS * 256);
    w.gpart = c.take<double>(n2 * SCF_KSPLIT_MAX);
    w.Fh = c.take<double>(n2 * std::max(1, p.diis));
    w.Eh = c.take<double>(n2 * std::max(1, p.diis));
    // the J/K workspace depends on the sizes only; the size query is given
    // placeholder addresses that it never dereferences
    static double placeholder[1];
    cd_jk_problem q = scf_jk_problem(p, placeholder, placeholder);
    q.row_pair = reinterpret_cast<const int64_t *>(placeholder);
    q.L = placeholder;
    q.n_vectors = reinterpret_cast<const int64_t *>(placeholder);
    q.C = placeholder;
    q.status = reinterpret_cast<int32_t *>(placeholder);
    size_t jb = 0;
    cd_status s = cd_query_jk(&q, 1, prec, &jb);
    if (s) return s;
    w.jk = c.take<char>(std::max<size_t>(1, jb));
    w.jk_bytes = std::max<size_t>(1, jb);
    bytes = c.off;
    return CD_OK;
}

static cd_status check_scf(const cd_scf_problem *p)
{
    if (!p) return fail(CD_ERR_INVALID_ARG, "null problem");
    if (p->n_basis < 1 || p->n_occ < 1 || p->n_occ > p->n_basis)
        return fail(CD_ERR_INVALID_ARG, "need 1 <= n_occ <= n_basis");
    if (p->max_iter < 1) return fail(CD_ERR_INVALID_ARG, "max_iter < 1");
    if (p->diis < 0 || p->diis > SCF_DIIS) return fail(CD_ERR_INVALID_ARG, "diis must be 0..%d", SCF_DIIS);
    if (!(p->e_tol >= 0.0) || !(p->d_tol >= 0.0))
        return fail(CD_ERR_INVALID_ARG, "tolerances must be >= 0");
    if ((int64_t)p->n_basis * p->n_basis > ((int64_t)1 << 31))
        return fail(CD_ERR_UNSUPPORTED, "basis too large");
    return CD_OK;
}

cd_status cd_query_scf(const cd_scf_problem *p, cd_precision prec, size_t *ws_bytes)
{
    if (!ws_bytes) return fail(CD_ERR_INVALID_ARG, "null ws_bytes");
    cd_status s = check_scf(p);
    if (s) return s;
    ScfWs w{};
    return scf_carve(*p, prec, nullptr, w, *ws_bytes);
}

cd_status cd_scf(cd_scf_problem *p, cd_precision prec, void *ws, size_t ws_bytes, void *stream)
{
    cd_status s = check_scf(p);
    if (s) return s;
    if (!p->S || !p->H || !p->C || !p->D || !p->F || !p->energies || !p->status ||
        !p->n_vectors || (p->n_rows > 0 && (!p->row_pair || !p->L)))
        return fail(CD_ERR_INVALID_ARG, "null pointer in SCF problem");
    ScfWs w{};
    size_t need = 0;
    if ((s = scf_carve(*p, prec, nullptr, w, need))) return s;
    if (need > ws_bytes || !ws)
        return fail(CD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if ((s = scf_carve(*p, prec, ws, w, need))) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int N = p->n_basis, O = p->n_occ;
    const int64_t n2 = (int64_t)N * N;
    const unsigned eb = (unsigned)blocks_of(n2, 256);
    const dim3 gg((unsigned)blocks_of(N, 64), (unsigned)blocks_of(N, 64));
    p->n_iter = 0;
    p->converged = 0;

    // k-splits of the N x N products: enough workgroups for the compute units
    const int tiles = (int)(blocks_of(N, 64) * blocks_of(N, 64));
    int ks = 1;
    while (ks < SCF_KSPLIT_MAX && tiles * (ks + 1) <= 256 && N / (ks + 1) >= 64) ++ks;
    const int kchunk = (int)(blocks_of(blocks_of(N, ks), SCF_TKC) * SCF_TKC);
    const dim3 gk(gg.x, gg.y, (unsigned)blocks_of(N, kchunk));
    auto gemm = [&](const double *A, const double *B, double *C) {
        if (gk.z == 1) {
            k_gemm_nn<<<gg, 256, 0, st>>>(N, A, B, C, N);
        } else {
            k_gemm_nn<<<gk, 256, 0, st>>>(N, A, B, w.gpart, kchunk);
            k_sum_split<<<eb, 256, 0, st>>>(n2, (int)gk.z, w.gpart, C);
        }
    };
    auto lincomb = [&](double *out, double a, const double *X, double b, const double *Y,
                       double c) { k_lincomb<<<eb, 256, 0, st>>>(N, out, a, X, b, Y, c); };
    // read 'n' reduction results back (synchronises the stream)
    double h[8];
    auto read = [&](int n) -> cd_status {
        cd_status r = check_launch("SCF kernels");
        if (r) return r;
        if (hipMemcpyAsync(h, w.red, sizeof(double) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(CD_ERR_DEVICE, "SCF read-back failed");
        return CD_OK;
    };

    k_fill_i32<<<1, 64, 0, st>>>(p->status, 1, 0);
    // grid-wide reductions: a fixed grid (the partition of the N^2 elements,
    // and so every sum, is the same on every call)
    const unsigned rb = (unsigned)std::min<int64_t>(256, blocks_of(n2, 256));
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(w.red);
    auto gershgorin = [&](const double *A) -> cd_status {
        k_gershgorin_init<<<1, 1, 0, st>>>(keys);
        k_gershgorin<<<(unsigned)blocks_of(N, 4), 256, 0, st>>>(N, A, keys);
        cd_status r = read(2);
        if (r) return r;
        unsigned long long kk[2];
        std::memcpy(kk, h, sizeof kk);
        h[0] = key_value(kk[0]);
        h[1] = key_value(kk[1]);
        return CD_OK;
    };
    auto maxabs = [&](const double *G, int minus_identity) -> cd_status {
        k_fill_f64<<<1, 64, 0, st>>>(w.red, 1, 0.0);
        k_maxabs<<<rb, 256, 0, st>>>(N, G, minus_identity, w.red);
        return read(1);
    };

    // ---- X = S^{-1/2}: coupled Newton-Schulz from Y = S / c, Z = I
    if ((s = gershgorin(p->S))) return s;
    const double c = h[1];
    if (!(c > 0.0) || !std::isfinite(c)) return fail(CD_ERR_NOT_PSD, "overlap bound %g", c);
    double *Y = w.A, *Z = w.B;
    lincomb(Y, 1.0 / c, p->S, 0.0, nullptr, 0.0);
    lincomb(Z, 0.0, p->S, 0.0, nullptr, 1.0);
    bool ns_ok = false;
    double prev = INFINITY;
    for (int it = 0; it < 200; ++it) {
        gemm(Z, Y, w.W1);
        if ((s = maxabs(w.W1, 1))) return s;
        const double err = h[0];
        if (!std::isfinite(err)) break;
        if (err < 1e-13 || (err < 1e-9 && err >= 0.5 * prev)) {
            ns_ok = true;
            break;
        }
        prev = err;
        lincomb(w.T, -0.5, w.W1, 0.0, nullptr, 1.5);
        gemm(Y, w.T, w.W2);
        std::swap(Y, w.W2);
        gemm(w.T, Z, w.W2);
        std::swap(Z, w.W2);
    }
    if (!ns_ok) return fail(CD_ERR_NOT_PSD, "Newton-Schulz for S^-1/2 did not converge");
    lincomb(w.X, 1.0 / std::sqrt(c), Z, 0.0, nullptr, 0.0);
    // the scratch pointers may have been swapped: keep A, B, W2 distinct from X
    double *bufs[3] = {Y, Z, w.W2};
    w.A = bufs[0];
    w.B = bufs[1];
    w.W2 = bufs[2];

    // ---- projector on the O lowest levels of Fm (in the S metric) into p->D
    auto purify = [&](const double *Fm) -> cd_status {
        double *Fo = w.A, *P = w.B, *P2 = w.T;
        gemm(w.X, Fm, w.W1);
        gemm(w.W1, w.X, Fo);
        cd_status r = gershgorin(Fo);
        if (r) return r;
        const double lo = h[0], hi = h[1];
        if (!(hi > lo)) return fail(CD_ERR_UNSUPPORTED, "degenerate Fock spectrum bounds");
        lincomb(P, -1.0 / (hi - lo), Fo, 0.0, nullptr, hi / (hi - lo));
        // the branch of each step is taken on the device from tr P; the host
        // reads the idempotency error tr P - tr P^2 once per chunk of steps
        // (steps past convergence leave an idempotent P as it is, up to rounding)
        constexpr int kChunk = 6;
        bool ok = false;
        double last = INFINITY;
        for (int it = 0; it < 400; it += kChunk) {
            for (int c = 0; c < kChunk; ++c) {
                gemm(P, P, P2);
                k_traces<<<1, 256, 0, st>>>(N, P, P2, w.red);
                k_tc2_step<<<eb, 256, 0, st>>>(N, P, P2, w.red, (double)O);
            }
            if ((r = read(2))) return r;
            const double e = std::fabs(h[0] - h[1]);
            if (!std::isfinite(e)) break;
            if (e < 1e-13 * O || (e < 1e-9 && e >= 0.5 * last)) {
                ok = true;
                break;
            }
            last = e;
        }
        if (!ok) return fail(CD_ERR_UNSUPPORTED, "purification did not converge (no gap?)");
        gemm(w.X, P, w.W1);
        gemm(w.W1, w.X, p->D);
        return CD_OK;
    };

    // Pulay extrapolation: history slots in age order and their error overlaps
    std::vector<int> order;
    double Bm[SCF_DIIS][SCF_DIIS] = {};
    auto extrapolate = [&](const double *G, double *Fx) -> cd_status {
        int slot;
        if ((int)order.size() < p->diis) {
            slot = (int)order.size();
        } else {
            slot = order.front();
            order.erase(order.begin());
        }
        order.push_back(slot);
        k_diis_store<<<eb, 256, 0, st>>>(N, G, p->F, w.Eh + slot * n2, w.Fh + slot * n2);
        DiisCoef co{};
        co.n = (int)order.size();
        for (int b = 0; b < co.n; ++b) co.slot[b] = order[b];
        k_diis_dots<<<dim3(rb, (unsigned)co.n), 256, 0, st>>>(n2, w.Eh + slot * n2, w.Eh, co,
                                                              w.part);
        k_sum_partials<<<(unsigned)co.n, 256, 0, st>>>((int)rb, w.part, 0.0, w.red);
        cd_status r = read(co.n);
        if (r) return r;
        for (int b = 0; b < co.n; ++b) Bm[slot][order[b]] = Bm[order[b]][slot] = h[b];
        // [B 1; 1^T 0] [c; -l] = [0; 1] by Gaussian elimination with partial pivoting
        const int n = co.n, m1 = n + 1;
        double A[SCF_DIIS + 1][SCF_DIIS + 2];
        for (int i = 0; i < m1; ++i) {
            for (int j = 0; j < m1; ++j)
                A[i][j] = (i < n && j < n) ? Bm[order[i]][order[j]] : (i == n && j == n ? 0.0 : 1.0);
            A[i][m1] = (i == n) ? 1.0 : 0.0;
        }
        for (int col = 0; col < m1; ++col) {
            int piv = col;
            for (int i = col + 1; i < m1; ++i)
                if (std::fabs(A[i][col]) > std::fabs(A[piv][col])) piv = i;
            if (A[piv][col] == 0.0) return fail(CD_ERR_UNSUPPORTED, "singular DIIS system");
            if (piv != col)
                for (int j = 0; j <= m1; ++j) std::swap(A[piv][j], A[col][j]);
            for (int i = col + 1; i < m1; ++i) {
                const double f = A[i][col] / A[col][col];
                for (int j = col; j <= m1; ++j) A[i][j] -= f * A[col][j];
            }
        }
        double x[SCF_DIIS + 1];
        for (int i = m1 - 1; i >= 0; --i) {
            double v = A[i][m1];
            for (int j = i + 1; j < m1; ++j) v -= A[i][j] * x[j];
            x[i] = v / A[i][i];
        }
        for (int b = 0; b < n; ++b) co.c[b] = x[b];
        k_diis_combine<<<eb, 256, 0, st>>>(n2, w.Fh, co, Fx);
        return check_launch("DIIS kernels");
    };

    if ((s = purify(p->H))) return s;
    cd_jk_problem q = scf_jk_problem(*p, w.J, w.K);
    double e_prev = 0.0;
    for (int k = 0; k < p->max_iter; ++k) {
        k_density_cholesky<<<1, DCH_T, 0, st>>>(N, O, p->D, w.W1, p->C, w.dres, p->status);
        if ((s = check_launch("density Cholesky"))) return s;
        if ((s = cd_build_jk(&q, 1, prec, 0, w.jk, w.jk_bytes, stream))) return s;
        k_fock_energy<<<rb, 256, 0, st>>>(N, p->H, w.J, w.K, p->D, p->F, w.part);
        k_sum_partials<<<1, 256, 0, st>>>((int)rb, w.part, p->e_charges, p->energies + k);
        gemm(p->F, p->D, w.W1);
        gemm(w.W1, p->S, w.W2);
        if ((s = maxabs(w.W2, 0))) return s;
        const double comm = h[0];
        double E = 0.0;
        int32_t dst = 0;
        if (hipMemcpy(&E, p->energies + k, sizeof E, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(&dst, p->status, sizeof dst, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(CD_ERR_DEVICE, "SCF read-back failed");
        if (dst != 0) return fail((cd_status)dst, "SCF iteration %d: device status %d", k, dst);
        p->n_iter = k + 1;
        if (k > 0 && std::fabs(E - e_prev) < p->e_tol && comm < p->d_tol) {
            p->converged = 1;
            break;
        }
        e_prev = E;
        if (k + 1 == p->max_iter) break;
        if (p->diis > 0) {
            if ((s = extrapolate(w.W2, w.W2))) return s;
            if ((s = purify(w.W2))) return s;
        } else if ((s = purify(p->F))) {
            return s;
        }
    }
    return CD_OK;
}

// Workgroups and rows per workgroup of the Hermitian decomposition.
static cd_status zcd_shape(int64_t n, int &G, int &R)
{
    DevInfo di;
    cd_status s = dev_info(di);
    if (s) return s;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_zcd, 256, 0) != hipSuccess)
        return fail(CD_ERR_DEVICE, "occupancy query failed");
    const int cap = std::min(kMaxGridBlocks, di.n_cu * std::max(1, nb));
    // at least 32 rows per workgroup: fewer workgroups make the per-vector
    // barrier cheaper, which pays until the rows' loads need the whole chip
    // (measured: 4096 rows 15.9 -> 15.2-15.4 ms with 128 workgroups; 8192 rows
    // keep 256)
    R = 32;
    while ((int64_t)R * cap < n && R < 256) R *= 2;
    if ((int64_t)R * cap < n) return fail(CD_ERR_UNSUPPORTED, "n = %lld rows exceed %d", (long long)n, R * cap);
    G = (int)std::max<int64_t>(1, blocks_of(n, R));
    return CD_OK;
}

static size_t zcd_ws_bytes()
{
    Carver c(nullptr);
    c.take<GridSync>(1);
    c.take<Nom>(2 * kMaxGridBlocks);
    return c.off;
}

cd_status cd_query_zdecompose(const cd_zproblem *p, size_t *ws_bytes)
{
    if (!p || !ws_bytes) return fail(CD_ERR_INVALID_ARG, "null argument");
    if (p->n < 0 || p->max_vectors < 0) return fail(CD_ERR_INVALID_ARG, "negative size");
    if (p->n > ((int64_t)1 << 31) - 1) return fail(CD_ERR_UNSUPPORTED, "n too large");
    *ws_bytes = zcd_ws_bytes();
    return CD_OK;
}

cd_status cd_zdecompose(const cd_zproblem *p, double tau, uint32_t flags, void *ws,
                        size_t ws_bytes, void *stream)
{
    size_t need = 0;
    cd_status s = cd_query_zdecompose(p, &need);
    if (s) return s;
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(CD_ERR_INVALID_ARG, "tau must be finite and >= 0");
    if (need > ws_bytes || !ws) return fail(CD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(CD_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    if (!p->n_vectors || !p->status) return fail(CD_ERR_INVALID_ARG, "null n_vectors/status");
    if (p->n > 0 && (!p->A || !p->diag || (p->max_vectors > 0 && (!p->L || !p->pivots))))
        return fail(CD_ERR_INVALID_ARG, "null pointer in Hermitian problem");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carver c(ws);
    GridSync *gs = c.take<GridSync>(1);
    Nom *part = c.take<Nom>(2 * kMaxGridBlocks);
    k_zcd_init<<<1, 256, 0, st>>>(gs, p->status, p->n_vectors);
    if ((s = check_launch("Hermitian init"))) return s;
    if (p->n > 0) {
        int G = 0, R = 0;
        if ((s = zcd_shape(p->n, G, R))) return s;
        ZcdParams Z{};
        Z.n = p->n;
        Z.A = static_cast<const double2 *>(p->A);
        Z.tau = tau;
        Z.max_vectors = p->max_vectors;
        Z.L = static_cast<double2 *>(p->L);
        Z.pivots = p->pivots;
        Z.D = p->diag;
        Z.n_vectors = p->n_vectors;
        Z.status = p->status;
        Z.gs = gs;
        Z.part = part;
        Z.G = G;
        Z.R = R;
        Z.spin_limit = 1u << 22;
        void *args[] = {&Z};
        if (hipLaunchCooperativeKernel((const void *)k_zcd, dim3(G), dim3(256), args, 0, st) != hipSuccess)
            return fail(CD_ERR_DEVICE, "Hermitian decomposition launch (%d workgroups) failed", G);
    }
    if (flags & CD_SYNC) {
        if (hipStreamSynchronize(st) != hipSuccess) return fail(CD_ERR_DEVICE, "stream synchronise failed");
        int32_t v = 0;
        if (hipMemcpy(&v, p->status, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(CD_ERR_DEVICE, "status copy failed");
        if (v != 0) return fail((cd_status)v, "Hermitian decomposition: device status %d", v);
    }
    return CD_OK;
}

cd_status cd_query_mp2(const cd_mp2_problem *probs, int32_t count, size_t *ws_bytes)
{
    if (count < 0 || (count > 0 && !probs) || !ws_bytes)
        return fail(CD_ERR_INVALID_ARG, "null argument");
    size_t tot = 0;
    for (int32_t i = 0; i < count; ++i) {
        const cd_mp2_problem &p = probs[i];
        if (p.n_occ < 0 || p.n_virt < 0 || p.max_vectors < 0)
            return fail(CD_ERR_INVALID_ARG, "negative size");
        Carver c(nullptr);
        c.take<double>(mp2_ws_doubles(p.n_occ, p.n_virt));
        tot += c.off;
    }
    *ws_bytes = tot;
    return CD_OK;
}

cd_status cd_mp2_energy(const cd_mp2_problem *probs, int32_t count, uint32_t flags, void *ws,
                        size_t ws_bytes, void *stream)
{
    size_t need = 0;
    cd_status s = cd_query_mp2(probs, count, &need);
    if (s) return s;
    if (need > ws_bytes || (need > 0 && !ws))
        return fail(CD_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *wbase = static_cast<char *>(ws);
    for (int32_t i = 0; i < count; ++i) {
        const cd_mp2_problem &p = probs[i];
        Carver c(wbase);
        double *w = c.take<double>(mp2_ws_doubles(p.n_occ, p.n_virt));
        wbase += c.off;
        if (!p.energy || !p.status || !p.n_vectors)
            return fail(CD_ERR_INVALID_ARG, "null pointer in mp2 problem %d", i);
        if (p.n_occ > 0 && p.n_virt > 0 && (!p.B || !p.e_occ || !p.e_virt))
            return fail(CD_ERR_INVALID_ARG, "null pointer in mp2 problem %d", i);
        Mp2Params Q{};
        Q.B = p.B;
        Q.max_vectors = p.max_vectors;
        Q.n_vectors = p.n_vectors;
        Q.O = p.n_occ;
        Q.V = p.n_virt;
        Q.eo = p.e_occ;
        Q.ev = p.e_virt;
        const int64_t T = blocks_of(p.n_virt, 64), TP = T * (T + 1) / 2;
        const int64_t NP = (int64_t)p.n_occ * (p.n_occ + 1) / 2;
        if (NP * TP > ((int64_t)1 << 31) - 8 || NP > ((int64_t)1 << 31) - 1)
            return fail(CD_ERR_UNSUPPORTED, "mp2 problem %d too large", i);
        Q.T = (int32_t)T;
        Q.TP = (int32_t)TP;
        Q.NP = (int32_t)NP;
        Q.per_xcd = blocks_of(NP * TP, 8);
        Q.partial = w;
        Q.pair_e = w + NP * TP;
        Q.pair_out = p.pair_energy;
        Q.energy = p.energy;
        Q.status = p.status;
        if (NP * TP > 0) k_mp2_tiles<<<(unsigned)(8 * Q.per_xcd), 256, 0, st>>>(Q);
        if (NP > 0) k_mp2_pairs<<<(unsigned)NP, 64, 0, st>>>(Q);
        k_mp2_total<<<1, 256, 0, st>>>(Q);
        if ((s = check_launch("mp2 kernels"))) return s;
    }
    if (flags & CD_SYNC) {
        if (hipStreamSynchronize(st) != hipSuccess)
            return fail(CD_ERR_DEVICE, "stream synchronise failed");
        for (int32_t i = 0; i < count; ++i) {
            int32_t v = 0;
            if (hipMemcpy(&v, probs[i].status, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
                return fail(CD_ERR_DEVICE, "status copy failed");
            if (v != 0) return fail((cd_status)v, "mp2 problem %d: device status %d", i, v);
        }
    }
    return CD_OK;
}

}  // extern "C"

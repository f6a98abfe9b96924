/*
 * cd.h -- C ABI of the MI355X (gfx950) Cholesky-decomposition library.
 *
 * The library computes, on the GPU, for molecules made of normalised s-type
 * Gaussians (paper: "Use of Cholesky decomposition in the CFOUR program
 * package"):
 *   cd_decompose  the threshold-truncated, fully pivoted Cholesky
 *                 decomposition of the two-electron-integral matrix over
 *                 composite pair indices (Sec. 2: initial diagonal, argmax
 *                 pivots, Eq. (subtr) vectors, Eq. (diag) diagonal update,
 *                 stop when max D < tau);
 *   cd_build_jk   the Coulomb and exchange matrices from the Cholesky vectors
 *                 and the occupied coefficients (Sec. 4.1: O(N^2 M) for J,
 *                 O(O N^2 M) for K);
 *   cd_transform  the AO->MO transform of the vectors (Sec. 4.1, CASSCF;
 *                 two-coefficient form of Sec. 6.2);
 *   cd_mp2_energy the second-order energy from transformed vectors (CD-based
 *                 MP2, Secs. 5 and 7);
 *   cd_one_electron, cd_scf  the SCF on Cholesky J/K (Sec. 4.1);
 *   cd_zdecompose the decomposition of a complex Hermitian matrix (Sec. 7).
 *
 * Conventions
 *   - Plain C, fixed-width integers; no C++ types or exceptions cross it.
 *   - Pointers documented as "device" are HIP device pointers; "host" are
 *     ordinary host memory.  The library never frees or retains caller
 *     memory.  Device inputs are read only.
 *   - Every call is stream ordered on the HIP stream passed as 'stream'
 *     (a hipStream_t, or NULL for the default stream) and asynchronous unless
 *     CD_SYNC is set or the function says otherwise.  Data-dependent results
 *     (number of vectors, status) are written to device memory.
 *   - Functions are ordered centre-major as given by the caller.  A "row" is
 *     a unique pair (mu >= nu) with packed index pq = mu(mu+1)/2 + nu; rows
 *     are kept iff sqrt(D1_row * max D1) >= schwarz (D1 = (mu nu|mu nu)) and
 *     are stored in ascending pq.
 *   - L is vector-major: L[K * n_rows + r] is vector K at row r.
 *   - Units: bohr, bohr^-2, hartree.
 *   - Return value: host-detectable errors (bad arguments, workspace too
 *     small, launch failure).  Device-detected conditions go to the
 *     problem's status word: CD_ERR_CAPACITY (max_vectors reached before the
 *     threshold), CD_ERR_NOT_PSD (a non-finite diagonal), CD_ERR_DEVICE (a
 *     device-side wait exceeded its bound).  With CD_SYNC the call
 *     synchronises the stream and folds status words into its return value.
 *   - cd_last_error() returns a thread-local message for the last error.
 */
#ifndef CD_MI355X_H
#define CD_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CD_OK = 0,
    CD_ERR_INVALID_ARG = 1,
    CD_ERR_WORKSPACE = 2,
    CD_ERR_CAPACITY = 3,
    CD_ERR_NOT_PSD = 4,
    CD_ERR_DEVICE = 5,
    CD_ERR_UNSUPPORTED = 6
} cd_status;

typedef enum {
    CD_FP64 = 0,   /* all contractions in FP64 */
    CD_FP32 = 1,   /* J/K contractions in FP32 (MFMA), FP64 across k-slabs */
    CD_BF16X3 = 2  /* J/K contractions on a 3-way BF16 split, 6 products, FP32
                      accumulation inside k-slabs, FP64 across slabs */
} cd_precision;

/* flags for cd_decomp_opts.flags and the J/K / transform calls */
#define CD_SYNC 1u /* synchronise the stream and fold device status into the return value */
/* cd_decompose only: continue finished decompositions to the (smaller) tau in
 * opts.  The pivot order of Sec. 2 does not depend on tau: the threshold only
 * decides where the loop stops (compare Table 5, where the number of vectors
 * grows as tau falls).  So a decomposition stopped at tau1 is the start of the
 * one at tau2 < tau1, and the loop can go on from where it stopped.  Each
 * problem's outputs must hold a decomposition of the same molecule with the
 * same schwarz and pivot_fn, written by cd_decompose into these same buffers
 * (row_pair, L, pivots, diag, n_vectors, status; pivot_values if given) and
 * ended with status CD_OK or CD_ERR_CAPACITY (a larger max_vectors may be
 * given after the caller moves the M1 vectors into a larger L: vector K is at
 * L + K * n_rows in any capacity).  n_rows and n_active come from cd_query at
 * the new tau; the workspace need not hold anything from the earlier call.
 * The first M1 vectors, their pivots and pivot values are not recomputed
 * (they stay bit for bit as they were); the selection continues from the
 * residuals in diag, and the all-row solve forms only the vectors from M1 on
 * and subtracts their squares from diag.  The result has the pivot sequence
 * of a direct run at the new tau; later vectors agree with that run to
 * rounding (the rounding order of the pivot selection's sums follows its
 * candidate batches, whose bounds depend on where the first run stopped).
 * A stored status other than CD_OK / CD_ERR_CAPACITY, or a stored count
 * outside [0, max_vectors], gives device status CD_ERR_INVALID_ARG and leaves
 * the outputs as they were. */
#define CD_RESUME 2u
/* cd_decompose only, for tests of the device error path: the setup replaces
 * the initial residual of the first active row by NaN, so the pivot selection
 * meets a non-finite diagonal (Sec. 2 needs a positive semidefinite matrix)
 * and reports CD_ERR_NOT_PSD in the problem's status word. */
#define CD_DEBUG_POISON_DIAG 4u

/* One molecule.  xyz and alpha are DEVICE pointers. */
typedef struct {
    int32_t n_basis;       /* N >= 0 */
    const double *xyz;     /* device [N][3], bohr */
    const double *alpha;   /* device [N], bohr^-2, > 0 */
    const uint8_t *pivot_fn; /* optional (may be NULL) device [N]: restricted candidates
                              (Sec. 6.2, the Cholesky basis taken from one block of rows).
                              When set, row (mu nu) may become a pivot only if pivot_fn[mu]
                              and pivot_fn[nu] are both nonzero; every row still gets its
                              vector elements and final residual, and the stop test runs over
                              the candidate rows only */
} cd_molecule;

/* Launch shapes of the decomposition kernels (0 in a field = the built-in
 * choice).  cd_autotune measures and returns one; cd_decompose takes one
 * through cd_decomp_opts.tuning. */
typedef struct {
    int32_t step2_row_tiles;   /* all-row solve: rows per workgroup in units of 16, 2..7 */
    int32_t step1_min_rows;    /* pivot selection: at least this many active rows per
                                  workgroup (fewer, fuller workgroups), 16..256 */
    int32_t step1_q;           /* pivot selection: candidates per batch, 8..64 (the pivot
                                  sequence is the same for every value) */
} cd_tuning;

typedef struct {
    double tau;            /* decomposition threshold (Sec. 2): stop when max D < tau; tau >= 0.
                              tau == 0 stops at max D <= n_rows * 2^-53 * max D1 */
    double schwarz;        /* row screening threshold, >= 0 (0 keeps all N(N+1)/2 rows) */
    uint32_t flags;        /* CD_SYNC, CD_RESUME, CD_DEBUG_POISON_DIAG */
    void *const *events;   /* optional (may be NULL): host array of 4 hipEvent_t that the call
                              records on 'stream' at the phase boundaries of the last problem:
                              [0] before the pair/diagonal setup, [1] before pivot selection,
                              [2] before the all-row substitution (k_step2; after the pivot
                              blocks' inverses and the solve's integral pass), [3] after it */
    int64_t *timeline;     /* optional (may be NULL): DEVICE buffer of 1 + 16 * timeline_cap int64
                              of device-clock (100 MHz) stamps of the last problem, for profiling.
                              [0]: number of candidate batches of the pivot selection;
                              [1 + 8 b + i]: batch b, stage i: 0 start, 1 nominations exchanged,
                              2 candidates chosen, 3 candidate columns formed, 4 columns
                              exchanged, 5 candidate block factored, 6 rows updated;
                              [1 + 8 cap + 8 k + i]: workgroup 0 of the all-row solve, 128-vector
                              block k, stage i: 0 start, 1 off-block product done and staged,
                              2 integrals subtracted, 3 substitution done, 4 residuals
                              updated, 5 stored */
    int64_t timeline_cap;  /* batches / blocks the timeline can hold */
    const cd_tuning *tuning; /* optional (may be NULL): host pointer to launch shapes */
    double eta;            /* span factor of the two-step first step (Sec. 3, Table 1), in [0, 1].
                              0 or 1: exact pivoting (Sec. 2: every pivot is the row of largest
                              residual).  0 < eta < 1: within a candidate batch a candidate is
                              also accepted while it is the largest remaining candidate and its
                              residual is >= eta times the batch's first pivot (the qualified set
                              of Table 1); the pivot sequence then differs from Sec. 2, every
                              final residual is still < tau */
} cd_decomp_opts;

/* Sizes of one decomposition problem, filled by cd_query. */
typedef struct {
    int64_t n_rows;        /* rows kept after screening */
    int64_t n_active;      /* rows with D1 >= tau that may be pivots (the only possible pivots;
                              candidate rows only when pivot_fn is set) */
    size_t ws_bytes;       /* device workspace cd_decompose needs for this problem
                              at the max_vectors passed to cd_query */
} cd_sizes;

/* Outputs of one decomposition (all DEVICE pointers, caller-allocated). */
typedef struct {
    cd_molecule mol;
    int64_t n_rows;        /* from cd_query */
    int64_t n_active;      /* from cd_query (same tau and schwarz) */
    int64_t max_vectors;   /* capacity of L and pivots */
    int64_t *row_pair;     /* [n_rows]   packed pair index of each row */
    double *L;             /* [max_vectors][n_rows] Cholesky vectors */
    int64_t *pivots;       /* [max_vectors] row index of pivot K (the Cholesky basis) */
    double *diag;          /* [n_rows] final residual diagonal (pivot rows zeroed when chosen) */
    int64_t *n_vectors;    /* [1] number of vectors M */
    int32_t *status;       /* [1] device status word (cd_status) */
    double *pivot_values;  /* optional (may be NULL): [max_vectors] d_K, the residual diagonal
                              at pivot P_K when vector K was formed (its square root is the
                              divisor of Sec. 2) */
} cd_problem;

/*
 * cd_query: screen the rows of each molecule on the device (blocking: it
 * synchronises 'stream') and report sizes and workspace.  'sizes' is a host
 * array of 'count' entries; 'max_vectors' is a host array of capacities.
 * Returns CD_ERR_INVALID_ARG for N < 0, tau < 0, schwarz < 0, null pointers.
 */
cd_status cd_query(const cd_molecule *mols, int32_t count, const cd_decomp_opts *opts,
                   const int64_t *max_vectors, cd_sizes *sizes, void *stream);

/*
 * cd_decompose: decompose 'count' molecules (host array 'probs') with the
 * workspace 'ws' (device, 256-byte aligned, ws_bytes >= the sum of cd_query's
 * ws_bytes; a misaligned ws gives CD_ERR_INVALID_ARG).
 * Asynchronous and free of host synchronisation unless CD_SYNC is set.  The
 * device recounts the rows; a count that differs from n_rows / n_active
 * gives status CD_ERR_DEVICE and no vectors.
 * The pivots follow Sec. 2 exactly: the pivot is the row of largest residual
 * diagonal (lowest row index among equal values; among the candidate rows when
 * the molecule's pivot_fn is set), the vector is
 * [(r|P) - sum_J L^J_r L^J_P] / sqrt(d_P) with d_P the tracked diagonal, the
 * pivot's own residual is set to zero, and the loop ends when max D < tau.
 * Rows whose D1 < tau can never be pivots and are only solved for at the
 * end (the two-step organisation of Sec. 3, with exact pivoting).
 * With count > 1 the per-problem setup runs on two library streams forked
 * from and joined back to 'stream' (ordering on 'stream' is kept on every
 * return, errors included; graph capture works).
 * opts->flags: CD_SYNC; CD_RESUME continues the decompositions already in the
 * outputs to opts->tau (see the flag); CD_DEBUG_POISON_DIAG (tests only).
 */
cd_status cd_decompose(const cd_problem *probs, int32_t count, const cd_decomp_opts *opts,
                       void *ws, size_t ws_bytes, void *stream);

/*
 * cd_decompose_noalloc: cd_decompose for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same problems, options, results and errors as
 * cd_decompose, with no workspace argument: the kernels use a static device
 * array of CD_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it
 * runs on until the process ends, and the call allocates nothing (no
 * hipMalloc or hipFree, no allocating library routine).  Problems whose
 * workspace (the sum of cd_query's ws_bytes for them) exceeds that size are
 * rejected with CD_ERR_WORKSPACE before any device work.  Every problem runs on
 * 'stream' (no library side streams).  All calls on one GPU share that GPU's
 * array, which keeps the last call's contents (the call initialises what it
 * needs): calls that overlap on one GPU (on different streams, or from
 * several threads without ordering) race and give wrong results; calls
 * ordered on one stream are safe.  The first call on a device also looks up
 * the array's device address there (once per device).
 */
#define CD_NOALLOC_SCRATCH_BYTES (128u << 20) /* 128 MiB */
cd_status cd_decompose_noalloc(const cd_problem *probs, int32_t count,
                               const cd_decomp_opts *opts, void *stream);

/*
 * cd_autotune: choose the launch shapes of cd_decompose for these problems by
 * measurement.  Blocking (synchronises 'stream').  It runs the decomposition
 * once per candidate shape, timing the pivot selection and the all-row solve
 * with HIP events: first every all-row-solve tile height (2..7 row tiles of
 * 16) with the built-in pivot-selection shape, then pivot-selection workgroups
 * of at least 16, 32, 48 or 64 active rows with the best tile height, then
 * batches of 32, 48 or 64 candidates with the best of those.  The fastest
 * shape is written to *best (host) and a last run with it leaves the
 * problems' outputs as cd_decompose would.  The library keeps the result for
 * the rest of the process, keyed by the device and the problems' shapes
 * (sizes, tau, screening, span factor, flags): a call with a shape seen before
 * runs the decomposition once with the kept result instead of measuring.
 * opts->tuning and opts->events are ignored.  Errors as cd_decompose; a device
 * status other than CD_OK in any run is returned as the result.
 */
cd_status cd_autotune(const cd_problem *probs, int32_t count, const cd_decomp_opts *opts,
                      void *ws, size_t ws_bytes, cd_tuning *best, void *stream);

/* One J/K build (all pointers DEVICE unless noted). */
typedef struct {
    int32_t n_basis;
    int64_t n_rows;
    int64_t max_vectors;
    const int64_t *row_pair;   /* [n_rows] from cd_decompose */
    const double *L;           /* [max_vectors][n_rows] */
    const int64_t *n_vectors;  /* [1] */
    int32_t n_occ;             /* O >= 0 */
    const double *C;           /* [N][O] occupied coefficients, D = C C^T */
    double *J;                 /* [N][N] out */
    double *K;                 /* [N][N] out */
    int32_t *status;           /* [1] */
    double *Lmo;               /* optional (may be NULL): [max_vectors][O][O] out,
                                  Lmo^P = C^T L^P C for P < M in FP64 (cd_transform with
                                  C1 = C2 = C) at every precision, formed from the FP64 half
                                  transform L^P C that K already needs */
} cd_jk_problem;

/* Workspace for cd_build_jk at the given precision (host-side, no device work). */
cd_status cd_query_jk(const cd_jk_problem *probs, int32_t count, cd_precision prec,
                      size_t *ws_bytes);

/*
 * cd_build_jk: J_{mu nu} = sum_P L^P_{mu nu} V^P, V^P = sum_{rho sigma} L^P_{rho sigma} D_{rho sigma};
 * K_{mu nu} = sum_P sum_i X^P_{i mu} X^P_{i nu}, X^P_{i mu} = sum_sigma L^P_{mu sigma} C_{sigma i}.
 * Screened pairs contribute nothing; J and K are symmetric and written in full.
 * Stream use: the work is ordered after what is already on 'stream', and
 * everything after the call on 'stream' is ordered after it.  In between, the
 * library runs parts of it (independent problems; for one problem the J chain
 * and the second half of Lmo) on two streams of its own, forked from and
 * joined back to 'stream' with events, so the call can be captured in a
 * graph.  Calls from several host threads enqueue one at a time.
 */
cd_status cd_build_jk(const cd_jk_problem *probs, int32_t count, cd_precision prec,
                      uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/* One AO->MO transform (all pointers DEVICE). */
typedef struct {
    int32_t n_basis;
    int64_t n_rows;
    int64_t max_vectors;
    const int64_t *row_pair;
    const double *L;
    const int64_t *n_vectors;
    int32_t p;                 /* columns of C1 */
    const double *C1;          /* [N][p] */
    int32_t q;                 /* columns of C2 */
    const double *C2;          /* [N][q] */
    double *Lmo;               /* [max_vectors][p][q] out: sum C1[mu][a] L^P_{mu nu} C2[nu][b] */
    int32_t *status;           /* [1] */
} cd_transform_problem;

cd_status cd_query_transform(const cd_transform_problem *probs, int32_t count, size_t *ws_bytes);

cd_status cd_transform(const cd_transform_problem *probs, int32_t count, uint32_t flags,
                       void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Second-order (MP2) energy from transformed vectors.  The CD-based MP2 of
 * Secs. 5 and 7 transforms the vectors to the molecular-orbital basis
 * (cd_transform with C1 = occupied, C2 = virtual coefficients) and contracts
 * them:
 *     (ia|jb) = sum_P B[P][i][a] B[P][j][b],
 *     e_ij = sum_{ab} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b),
 *     E = sum_{ij} e_ij
 * (the textbook closed-shell energy; the denominators must not vanish).
 * FP64 throughout.  Asynchronous; cd_query_mp2 gives the workspace size.
 * Device status: CD_ERR_INVALID_ARG when *n_vectors is outside
 * [0, max_vectors] (then E = 0).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_occ;             /* O >= 0 */
    int32_t n_virt;            /* V >= 0 */
    int64_t max_vectors;       /* leading dimension of B */
    const int64_t *n_vectors;  /* [1] M (e.g. written by cd_decompose) */
    const double *B;           /* [max_vectors][O][V] transformed vectors (cd_transform's Lmo) */
    const double *e_occ;       /* [O] occupied orbital energies, hartree */
    const double *e_virt;      /* [V] virtual orbital energies, hartree */
    double *energy;            /* [1] out: E */
    double *pair_energy;       /* optional (may be NULL) [O][O] out: e_ij */
    int32_t *status;           /* [1] */
} cd_mp2_problem;

cd_status cd_query_mp2(const cd_mp2_problem *probs, int32_t count, size_t *ws_bytes);

cd_status cd_mp2_energy(const cd_mp2_problem *probs, int32_t count, uint32_t flags, void *ws,
                        size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * SCF on Cholesky J/K (Sec. 4.1): the one-electron integrals and a
 * closed-shell Roothaan-Hall loop whose J and K come from cd_build_jk.
 * ------------------------------------------------------------------------ */
typedef struct {
    cd_molecule mol;           /* the basis (pivot_fn is ignored) */
    int32_t n_charges;         /* point charges, >= 0 */
    const double *charge_xyz;  /* device [n_charges][3], bohr */
    const double *charge;      /* device [n_charges] */
    double *S;                 /* out, device [N][N]: overlap */
    double *H;                 /* out, device [N][N]: kinetic energy + attraction to the charges */
} cd_one_electron_problem;

/* S and H in closed form for normalised s functions (textbook formulas with
 * F0).  Asynchronous unless flags has CD_SYNC. */
cd_status cd_one_electron(const cd_one_electron_problem *p, uint32_t flags, void *stream);

typedef struct {
    /* Cholesky vectors, as in cd_jk_problem (device) */
    int32_t n_basis;
    int64_t n_rows;
    int64_t max_vectors;
    const int64_t *row_pair;
    const double *L;
    const int64_t *n_vectors;
    int32_t n_occ;             /* O doubly occupied orbitals, 1 <= O <= N */
    const double *S;           /* device [N][N] overlap */
    const double *H;           /* device [N][N] one-electron Hamiltonian */
    double e_charges;          /* host value added to every energy (charge repulsion) */
    int32_t max_iter;          /* >= 1 */
    double e_tol;              /* converged when |E_k - E_(k-1)| < e_tol ... */
    double d_tol;              /* ... and max |F D S - S D F| < d_tol */
    int32_t diis;              /* Pulay extrapolation over the last 'diis' Fock matrices, 0..8
                                  (0: plain Roothaan steps) */
    double *C;                 /* out, device [N][O]: D = C C^T (pivoted Cholesky factor of D) */
    double *D;                 /* out, device [N][N]: density of the last iteration */
    double *F;                 /* out, device [N][N]: F(D) = H + 2 J(D) - K(D) */
    double *energies;          /* out, device [max_iter]: E_k = tr(D_k (H + F_k)) + e_charges */
    int32_t *status;           /* device [1] */
    int32_t n_iter;            /* out (host field): energies written */
    int32_t converged;         /* out (host field): 1 if the tolerances were met */
} cd_scf_problem;

/* Workspace bytes of cd_scf (host-side, no device work). */
cd_status cd_query_scf(const cd_scf_problem *p, cd_precision prec, size_t *ws_bytes);

/*
 * cd_scf: D_0 projects on the O lowest solutions of H C = S C e (core
 * guess); iteration k builds J and K of D_k = C_k C_k^T from the vectors at
 * precision 'prec', F_k = H + 2 J - K and E_k, and stops on convergence;
 * otherwise D_(k+1) projects on the O lowest solutions of F C = S C e, where F
 * is F_k or, with diis > 0, Pulay's extrapolation sum_i c_i F_i (sum c_i = 1,
 * minimal |sum c_i e_i| over the stored commutators e_i).  The
 * projector comes from trace-correcting purification of X F X with
 * X = S^(-1/2) (Newton-Schulz), not from a diagonalisation.  Blocking: the
 * host reads the convergence figures.  Errors: CD_ERR_INVALID_ARG (sizes,
 * pointers), CD_ERR_NOT_PSD (the orthogonaliser does not converge: S is not
 * positive definite to working precision), CD_ERR_UNSUPPORTED (purification
 * does not converge: no gap between the O-th and (O+1)-th level), and the
 * errors of cd_build_jk.
 */
cd_status cd_scf(cd_scf_problem *p, cd_precision prec, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Hermitian decomposition (Sec. 7, finite magnetic field): the integrals over
 * field-dependent orbitals are complex and the matrix is Hermitian positive
 * semidefinite with a real diagonal.  Sec. 2 in complex algebra, on a matrix
 * given explicitly:
 *     P_K = argmax_r D_r (lowest r on ties), d_K = D_(P_K), stop when d_K < tau
 *     (tau == 0: also when d_K <= n 2^-53 max_r A_rr),
 *     L^K_r = [A_(r P_K) - sum_(J<K) L^J_r conj(L^J_(P_K))] / sqrt(d_K),
 *     D_r -= |L^K_r|^2, D_(P_K) = 0,
 * so A_rs ~ sum_K L^K_r conj(L^K_s).  Complex values are (re, im) pairs of
 * doubles.  Device status: CD_ERR_CAPACITY (max_vectors reached before the
 * threshold), CD_ERR_NOT_PSD (a non-finite or non-positive pivot),
 * CD_ERR_DEVICE (a device-side wait exceeded its bound).
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;                 /* rows, 0 <= n < 2^31 (and n <= 256 x the resident workgroups) */
    const void *A;             /* device [n][n] complex double, Hermitian (only A read) */
    int64_t max_vectors;       /* capacity of L and pivots */
    void *L;                   /* out, device [max_vectors][n] complex double */
    int64_t *pivots;           /* out, device [max_vectors] */
    double *diag;              /* out, device [n] final residual diagonal */
    int64_t *n_vectors;        /* out, device [1] */
    int32_t *status;           /* out, device [1] */
} cd_zproblem;

/* Workspace bytes of cd_zdecompose (host-side). */
cd_status cd_query_zdecompose(const cd_zproblem *p, size_t *ws_bytes);

/* One persistent cooperative launch; asynchronous unless flags has CD_SYNC.
 * ws: device, 256-byte aligned, at least cd_query_zdecompose's bytes. */
cd_status cd_zdecompose(const cd_zproblem *p, double tau, uint32_t flags, void *ws,
                        size_t ws_bytes, void *stream);

/* Thread-local message describing the last error returned on this thread. */
const char *cd_last_error(void);

/* Library version string. */
const char *cd_version(void);

#ifdef __cplusplus
}
#endif
#endif

/*
 * CPU oracle for the Cholesky-decomposition path: plain, slow, FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes (paper: "Use of Cholesky decomposition in the CFOUR
 * program package"):
 *   - electron-repulsion integrals over normalised s-type Gaussians (the
 *     paper evaluates ERIs by the McMurchie-Davidson scheme, Sec. 7; for s
 *     functions that scheme collapses to the textbook closed form with the
 *     zeroth-order Boys function, which is what is written out here);
 *   - the threshold-truncated, fully pivoted Cholesky decomposition of the
 *     ERI matrix over composite pair indices, step by step as Sec. 2 states
 *     it (initial diagonal, argmax pivot, Eq. (subtr) for the vector,
 *     Eq. (diag) for the diagonal, stop when max D < tau);
 *   - the Coulomb and exchange matrices from the Cholesky vectors (Sec. 4.1
 *     states their O(N^2 M) and O(O N^2 M) cost; the formulas are the
 *     standard J and K with (mu nu|rho sigma) ~ sum_P L^P_{mu nu} L^P_{rho sigma}
 *     inserted), and the same J and K from exact integrals (brute force);
 *   - the AO->MO transform of the vectors (Sec. 4.1, CASSCF; two-coefficient
 *     form of Sec. 6.2);
 *   - the closed-shell second-order (MP2) energy from transformed vectors
 *     (CD-based MP2 of Secs. 5 and 7; the textbook energy expression);
 *   - the threshold-truncated, fully pivoted Cholesky decomposition of a
 *     complex Hermitian positive semidefinite matrix (the finite-field case
 *     of Sec. 7: complex integrals, a real diagonal, complex vectors with
 *     A ~ sum_K L_K L_K^H), given the matrix explicitly;
 *   - one-electron integrals over the same functions (overlap, kinetic
 *     energy, attraction to point charges) and the repulsion of the charges,
 *     the ingredients of the SCF of Sec. 4.1 besides J and K (textbook
 *     closed forms for s functions).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   ties in the argmax go to the lowest row index; the divisor is the square
 *   root of the tracked diagonal D at the pivot; the pivot's own diagonal is
 *   set to exactly zero after its vector is formed; the loop stops when
 *   max D < tau (strict), and for tau <= 0 additionally when
 *   max D <= n * 2^-53 * max D^1; rows are kept iff
 *   sqrt(D^1_row * max D^1) >= schwarz, in ascending packed order
 *   pq = mu(mu+1)/2 + nu (mu >= nu).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---- Boys function of order zero -------------------------------------- */
/* F0(T) = int_0^1 exp(-T t^2) dt = (1/2) sqrt(pi/T) erf(sqrt(T)), F0(0) = 1. */
double or_boys0(double T)
{
    if (T == 0.0) return 1.0;
    double x = sqrt(T);
    return 0.5 * sqrt(M_PI / T) * erf(x);
}

/* ---- pair data ---------------------------------------------------------- */
/* Product of two normalised s primitives g = (2a/pi)^{3/4} exp(-a |r-A|^2):
 *   p = a_mu + a_nu,  P = (a_mu A_mu + a_nu A_nu) / p,
 *   E = N_mu N_nu exp(-a_mu a_nu / p |A_mu - A_nu|^2). */
static void pair_data(const double *xyz, const double *alpha, int mu, int nu,
                      double *p, double P[3], double *E)
{
    double a = alpha[mu], b = alpha[nu];
    double s = a + b;
    double r2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double d = xyz[3 * mu + k] - xyz[3 * nu + k];
        r2 += d * d;
        P[k] = (a * xyz[3 * mu + k] + b * xyz[3 * nu + k]) / s;
    }
    double na = pow(2.0 * a / M_PI, 0.75);
    double nb = pow(2.0 * b / M_PI, 0.75);
    *p = s;
    *E = na * nb * exp(-a * b / s * r2);
}

/* (mu nu | sg rh) = 2 pi^{5/2} / (p q sqrt(p+q)) E_{mu nu} E_{sg rh} F0(T),
 * T = p q / (p+q) |P - Q|^2. */
double or_eri(const double *xyz, const double *alpha, int mu, int nu, int sg, int rh)
{
    double p, q, P[3], Q[3], E1, E2;
    pair_data(xyz, alpha, mu, nu, &p, P, &E1);
    pair_data(xyz, alpha, sg, rh, &q, Q, &E2);
    double r2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double d = P[k] - Q[k];
        r2 += d * d;
    }
    double T = p * q / (p + q) * r2;
    return 2.0 * pow(M_PI, 2.5) / (p * q * sqrt(p + q)) * E1 * E2 * or_boys0(T);
}

static void unpack(int64_t pq, int *mu, int *nu)
{
    /* largest mu with mu(mu+1)/2 <= pq */
    int m = (int)floor((sqrt(8.0 * (double)pq + 1.0) - 1.0) * 0.5);
    while ((int64_t)m * (m + 1) / 2 > pq) --m;
    while ((int64_t)(m + 1) * (m + 2) / 2 <= pq) ++m;
    *mu = m;
    *nu = (int)(pq - (int64_t)m * (m + 1) / 2);
}

void or_unpack_pair(int64_t pq, int32_t *mu, int32_t *nu)
{
    int a, b;
    unpack(pq, &a, &b);
    *mu = a;
    *nu = b;
}

/* Diagonal (mu nu|mu nu) of every unique pair, in packed order. */
void or_diagonal_all(int N, const double *xyz, const double *alpha, double *D1)
{
    int64_t k = 0;
    for (int mu = 0; mu < N; ++mu)
        for (int nu = 0; nu <= mu; ++nu)
            D1[k++] = or_eri(xyz, alpha, mu, nu, mu, nu);
}

/* Screened row list.  Returns the row count; row_pair must hold N(N+1)/2. */
int64_t or_rows(int N, const double *xyz, const double *alpha, double schwarz,
                int64_t *row_pair, double *D1max_out)
{
    int64_t np = (int64_t)N * (N + 1) / 2;
    double *D1 = (double *)malloc(sizeof(double) * (size_t)(np ? np : 1));
    or_diagonal_all(N, xyz, alpha, D1);
    double mx = 0.0;
    for (int64_t k = 0; k < np; ++k)
        if (D1[k] > mx) mx = D1[k];
    int64_t n = 0;
    for (int64_t k = 0; k < np; ++k)
        if (sqrt(D1[k] * mx) >= schwarz) row_pair[n++] = k;
    free(D1);
    if (D1max_out) *D1max_out = mx;
    return n;
}

static double eri_rows(const double *xyz, const double *alpha, int64_t pa, int64_t pb)
{
    int a, b, c, d;
    unpack(pa, &a, &b);
    unpack(pb, &c, &d);
    return or_eri(xyz, alpha, a, b, c, d);
}

/* Explicit ERI matrix over the given rows, [n][n] row-major (small cases). */
void or_eri_matrix(const double *xyz, const double *alpha, int64_t n,
                   const int64_t *row_pair, double *A)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            A[i * n + j] = eri_rows(xyz, alpha, row_pair[i], row_pair[j]);
}

/*
 * Fully pivoted, threshold-truncated Cholesky decomposition (Sec. 2).
 *
 *   D^1_r = (r|r)
 *   loop K = 0, 1, ...:
 *     P_K = argmax_r D_r   (lowest r on ties)      d_K = D_{P_K}
 *     stop if d_K < tau   (or d_K <= floor when tau <= 0)
 *     L^K_r = [ (r|P_K) - sum_{J<K} L^J_r L^J_{P_K} ] / sqrt(d_K)     Eq. (subtr)
 *     D_r  -= (L^K_r)^2                                                Eq. (diag)
 *     D_{P_K} = 0
 *
 * L is vector-major: L[K * n + r].  If 'given' is non-NULL the pivots are
 * taken from it instead (replay); each given pivot is checked to be a valid
 * argmax within 'tie_tol' (D_given >= max D - tie_tol); the index of the
 * first violation is written to *bad (or -1).  Replay stops after n_given
 * pivots or at the threshold, whichever comes first.
 *
 * If 'cand' is non-NULL, only rows with cand[r] != 0 may become pivots
 * (restricted candidates, Sec. 6.2: the Cholesky basis chosen from one block
 * of rows only): the argmax and the stop test run over those rows, and every
 * row still gets its elements of each vector and its residual D.
 *
 * Returns 0 on success, 1 if max_vectors was reached before the threshold,
 * 2 if a pivot value was not positive and finite.
 */
int or_decompose(const double *xyz, const double *alpha, int64_t n, const int64_t *row_pair,
                 double tau, int64_t max_vectors, double *L, int64_t *pivots,
                 double *dpiv, double *D, int64_t *M_out,
                 const int64_t *given, int64_t n_given, double tie_tol, int64_t *bad,
                 const unsigned char *cand)
{
    int rc = 0;
    int64_t M = 0;
    if (bad) *bad = -1;
    double d1max = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        D[r] = eri_rows(xyz, alpha, row_pair[r], row_pair[r]);
        if (D[r] > d1max) d1max = D[r];
    }
    double floor_tol = (double)n * ldexp(1.0, -53) * d1max;
    double *col = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    for (;;) {
        int64_t piv = -1;
        double d = -INFINITY;
        for (int64_t r = 0; r < n; ++r)
            if ((!cand || cand[r]) && D[r] > d) { d = D[r]; piv = r; }
        if (n == 0 || d < tau) break;
        if (tau <= 0.0 && d <= floor_tol) break;
        if (given) {
            if (M >= n_given) break;
            int64_t g = given[M];
            if (g < 0 || g >= n || (cand && !cand[g])) { if (bad && *bad < 0) *bad = M; break; }
            if (D[g] < d - tie_tol && bad && *bad < 0) *bad = M;
            piv = g;
            d = D[g];
            if (d < tau) break;
        }
        if (M >= max_vectors) { rc = 1; break; }
        if (!(d > 0.0) || !isfinite(d)) { rc = 2; break; }
        int64_t P = row_pair[piv];
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r)
            col[r] = eri_rows(xyz, alpha, row_pair[r], P);
        for (int64_t J = 0; J < M; ++J) {
            const double *LJ = L + J * n;
            double lp = LJ[piv];
#pragma omp parallel for schedule(static)
            for (int64_t r = 0; r < n; ++r)
                col[r] -= LJ[r] * lp;
        }
        double s = sqrt(d);
        double *LK = L + M * n;
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            LK[r] = col[r] / s;
            D[r] -= LK[r] * LK[r];
        }
        D[piv] = 0.0;
        pivots[M] = piv;
        dpiv[M] = d;
        ++M;
    }
    free(col);
    *M_out = M;
    return rc;
}

/* Density D = C C^T, C [N][O] row-major. */
static void density(int N, int O, const double *C, double *Dm)
{
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            double s = 0.0;
            for (int i = 0; i < O; ++i) s += C[a * O + i] * C[b * O + i];
            Dm[a * N + b] = s;
        }
}

/* Unpack vector P into a symmetric N x N matrix (zero for screened pairs). */
static void unpack_vector(int N, int64_t n, const int64_t *row_pair, const double *LP, double *S)
{
    memset(S, 0, sizeof(double) * (size_t)N * N);
    for (int64_t r = 0; r < n; ++r) {
        int mu, nu;
        unpack(row_pair[r], &mu, &nu);
        S[mu * N + nu] = LP[r];
        S[nu * N + mu] = LP[r];
    }
}

/*
 * J and K from the Cholesky vectors, D = C C^T:
 *   J_{mu nu} = sum_P L^P_{mu nu} sum_{sg rh} L^P_{sg rh} D_{sg rh}
 *   K_{mu nu} = sum_P sum_i X^P_{i mu} X^P_{i nu},  X^P_{i mu} = sum_sg L^P_{mu sg} C_{sg i}
 * J, K are [N][N] row-major.
 */
void or_jk_cd(int N, int64_t n, const int64_t *row_pair, const double *L, int64_t M,
              const double *C, int O, double *J, double *K)
{
    double *Dm = (double *)malloc(sizeof(double) * (size_t)N * N);
    density(N, O, C, Dm);
    memset(J, 0, sizeof(double) * (size_t)N * N);
    memset(K, 0, sizeof(double) * (size_t)N * N);
#pragma omp parallel
    {
        double *S = (double *)malloc(sizeof(double) * (size_t)N * N);
        double *X = (double *)malloc(sizeof(double) * (size_t)N * (O ? O : 1));
        double *Jt = (double *)calloc((size_t)N * N, sizeof(double));
        double *Kt = (double *)calloc((size_t)N * N, sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t P = 0; P < M; ++P) {
            unpack_vector(N, n, row_pair, L + P * n, S);
            double v = 0.0;
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b) v += S[a * N + b] * Dm[a * N + b];
            for (int a = 0; a < N * N; ++a) Jt[a] += S[a] * v;
            for (int mu = 0; mu < N; ++mu)
                for (int i = 0; i < O; ++i) {
                    double s = 0.0;
                    for (int sg = 0; sg < N; ++sg) s += S[mu * N + sg] * C[sg * O + i];
                    X[mu * O + i] = s;
                }
            for (int mu = 0; mu < N; ++mu)
                for (int nu = 0; nu < N; ++nu) {
                    double s = 0.0;
                    for (int i = 0; i < O; ++i) s += X[mu * O + i] * X[nu * O + i];
                    Kt[mu * N + nu] += s;
                }
        }
#pragma omp critical
        {
            for (int a = 0; a < N * N; ++a) { J[a] += Jt[a]; K[a] += Kt[a]; }
        }
        free(S); free(X); free(Jt); free(Kt);
    }
    free(Dm);
}

/* Brute-force J_{mu nu} = sum (mu nu|sg rh) D_{sg rh},
 * K_{mu nu} = sum (mu sg|nu rh) D_{sg rh}, from exact integrals. O(N^4). */
void or_jk_exact(int N, const double *xyz, const double *alpha, const double *C, int O,
                 double *J, double *K)
{
    double *Dm = (double *)malloc(sizeof(double) * (size_t)N * N);
    density(N, O, C, Dm);
#pragma omp parallel for schedule(dynamic, 1)
    for (int mu = 0; mu < N; ++mu)
        for (int nu = 0; nu < N; ++nu) {
            double sj = 0.0, sk = 0.0;
            for (int sg = 0; sg < N; ++sg)
                for (int rh = 0; rh < N; ++rh) {
                    sj += or_eri(xyz, alpha, mu, nu, sg, rh) * Dm[sg * N + rh];
                    sk += or_eri(xyz, alpha, mu, sg, nu, rh) * Dm[sg * N + rh];
                }
            J[mu * N + nu] = sj;
            K[mu * N + nu] = sk;
        }
    free(Dm);
}

/* E2 = 2 tr(D J) - tr(D K): closed-shell two-electron energy for doubly
 * occupied C, D = C C^T. */
double or_e2(int N, const double *C, int O, const double *J, const double *K)
{
    double *Dm = (double *)malloc(sizeof(double) * (size_t)N * N);
    density(N, O, C, Dm);
    double e = 0.0;
    for (int a = 0; a < N * N; ++a) e += Dm[a] * (2.0 * J[a] - K[a]);
    free(Dm);
    return e;
}

/* AO->MO transform: Lmo[P][a][b] = sum_{mu nu} C1[mu][a] L^P_{mu nu} C2[nu][b]. */
void or_transform(int N, int64_t n, const int64_t *row_pair, const double *L, int64_t M,
                  const double *C1, int p, const double *C2, int q, double *Lmo)
{
#pragma omp parallel
    {
        double *S = (double *)malloc(sizeof(double) * (size_t)N * N);
        double *T = (double *)malloc(sizeof(double) * (size_t)N * (q ? q : 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t P = 0; P < M; ++P) {
            unpack_vector(N, n, row_pair, L + P * n, S);
            for (int mu = 0; mu < N; ++mu)
                for (int b = 0; b < q; ++b) {
                    double s = 0.0;
                    for (int nu = 0; nu < N; ++nu) s += S[mu * N + nu] * C2[nu * q + b];
                    T[mu * q + b] = s;
                }
            double *out = Lmo + P * (int64_t)p * q;
            for (int a = 0; a < p; ++a)
                for (int b = 0; b < q; ++b) {
                    double s = 0.0;
                    for (int mu = 0; mu < N; ++mu) s += C1[mu * p + a] * T[mu * q + b];
                    out[a * q + b] = s;
                }
        }
        free(S); free(T);
    }
}

/* Closed-shell second-order (MP2) pair energy from transformed vectors,
 * B[P][i][a] = sum_{mu nu} C_occ[mu][i] L^P_{mu nu} C_virt[nu][a] (the
 * CD-based MP2 of Secs. 5 and 7 of the paper; the energy expression is the
 * textbook closed-shell one, not printed in the paper):
 *   (ia|jb) = sum_P B[P][i][a] B[P][j][b],
 *   e_ij = sum_{ab} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b).
 * The total energy is sum over all ordered pairs (i, j). */
double or_mp2_pair(int64_t M, int O, int V, const double *B, const double *eo,
                   const double *ev, int i, int j)
{
    if (V <= 0) return 0.0;
    double *W = (double *)malloc(sizeof(double) * (size_t)V * V);
#pragma omp parallel for schedule(static)
    for (int a = 0; a < V; ++a)
        for (int b = 0; b < V; ++b) {
            double s = 0.0;
            for (int64_t P = 0; P < M; ++P)
                s += B[(P * O + i) * V + a] * B[(P * O + j) * V + b];
            W[a * V + b] = s;
        }
    double e = 0.0;
    for (int a = 0; a < V; ++a)
        for (int b = 0; b < V; ++b) {
            const double w = W[a * V + b];
            e += w * (2.0 * w - W[b * V + a]) / (eo[i] + eo[j] - ev[a] - ev[b]);
        }
    free(W);
    return e;
}

/* All pair energies (pair[i * O + j]) and their sum. */
double or_mp2(int64_t M, int O, int V, const double *B, const double *eo, const double *ev,
              double *pair)
{
    double e = 0.0;
    for (int i = 0; i < O; ++i)
        for (int j = 0; j < O; ++j) {
            const double s = or_mp2_pair(M, O, V, B, eo, ev, i, j);
            if (pair) pair[i * O + j] = s;
            e += s;
        }
    return e;
}

/* ---- one-electron integrals (SCF, Sec. 4.1) ------------------------------ */
/* For normalised s primitives a, b (exponents x_a, x_b, centres A, B):
 *   S_ab = N_a N_b (pi/p)^{3/2} exp(-x_a x_b / p |A-B|^2),   p = x_a + x_b
 *   T_ab = m (3 - 2 m |A-B|^2) S_ab,                          m = x_a x_b / p
 *   V_ab = -sum_C Z_C (2 pi / p) N_a N_b exp(-m |A-B|^2) F0(p |P-C|^2)
 * with P the Gaussian product centre.  Outputs are [N][N] row-major. */
void or_one_electron(int N, const double *xyz, const double *alpha, int nc,
                     const double *cxyz, const double *Z, double *S, double *T, double *V)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            double p, P[3], E;
            pair_data(xyz, alpha, a, b, &p, P, &E);
            double m = alpha[a] * alpha[b] / p, r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double d = xyz[3 * a + k] - xyz[3 * b + k];
                r2 += d * d;
            }
            double s = E * pow(M_PI / p, 1.5);
            double v = 0.0;
            for (int c = 0; c < nc; ++c) {
                double pc2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    double d = P[k] - cxyz[3 * c + k];
                    pc2 += d * d;
                }
                v -= Z[c] * 2.0 * M_PI / p * E * or_boys0(p * pc2);
            }
            S[a * N + b] = s;
            T[a * N + b] = m * (3.0 - 2.0 * m * r2) * s;
            V[a * N + b] = v;
        }
}

/* Repulsion of the point charges, sum_{C<D} Z_C Z_D / |C - D|. */
double or_charge_repulsion(int nc, const double *cxyz, const double *Z)
{
    double e = 0.0;
    for (int c = 0; c < nc; ++c)
        for (int d = 0; d < c; ++d) {
            double r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double t = cxyz[3 * c + k] - cxyz[3 * d + k];
                r2 += t * t;
            }
            e += Z[c] * Z[d] / sqrt(r2);
        }
    return e;
}

/* ---- Hermitian decomposition (Sec. 7) ----------------------------------- */
/*
 * A: [n][n] complex, Hermitian positive semidefinite (row-major).  Sec. 2
 * with complex algebra:
 *   D_r = A_rr (real);  P_K = argmax_r D_r (lowest r on ties);  d_K = D_{P_K}
 *   stop if d_K < tau (or d_K <= n 2^-53 max D when tau <= 0)
 *   L^K_r = [ A_{r P_K} - sum_{J<K} L^J_r conj(L^J_{P_K}) ] / sqrt(d_K)
 *   D_r -= |L^K_r|^2;  D_{P_K} = 0
 * so that A_rs ~ sum_K L^K_r conj(L^K_s).  L is vector-major [K][n].
 * Returns 0, or 1 at capacity, 2 for a non-positive / non-finite pivot.
 */
int or_zdecompose(int64_t n, const double complex *A, double tau, int64_t max_vectors,
                  double complex *L, int64_t *pivots, double *D, int64_t *M_out)
{
    int rc = 0;
    int64_t M = 0;
    double dmax = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        D[r] = creal(A[r * n + r]);
        if (D[r] > dmax) dmax = D[r];
    }
    const double floor_tol = (double)n * ldexp(1.0, -53) * dmax;
    for (;;) {
        int64_t piv = -1;
        double d = -INFINITY;
        for (int64_t r = 0; r < n; ++r)
            if (D[r] > d) { d = D[r]; piv = r; }
        if (n == 0 || d < tau) break;
        if (tau <= 0.0 && d <= floor_tol) break;
        if (M >= max_vectors) { rc = 1; break; }
        if (!(d > 0.0) || !isfinite(d)) { rc = 2; break; }
        const double s = sqrt(d);
        double complex *LK = L + M * n;
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            double complex v = A[r * n + piv];
            for (int64_t J = 0; J < M; ++J) v -= L[J * n + r] * conj(L[J * n + piv]);
            LK[r] = v / s;
        }
        for (int64_t r = 0; r < n; ++r) D[r] -= creal(LK[r]) * creal(LK[r]) + cimag(LK[r]) * cimag(LK[r]);
        D[piv] = 0.0;
        pivots[M] = piv;
        ++M;
    }
    *M_out = M;
    return rc;
}


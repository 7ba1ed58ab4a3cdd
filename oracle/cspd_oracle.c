/*
 * FP64 CPU oracle for full OMP and cross-scale (zero-tree) OMP.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or helper with the
 * HIP library.
 *
 * What it computes (Saragadam, Li, Sankaranarayanan, "Cross-Scale Predictive
 * Dictionaries"):
 *   - Algorithm 1 (orthogonal matching pursuit): for n = 1..K pick the atom
 *     closest in angle to the residue (proxy), merge it into the support,
 *     solve the least-squares problem on the support (projection) and form
 *     the new residue.
 *   - Section III-C / Algorithm 2 (zero-tree OMP): problem (P_low) is OMP on
 *     y against the effective coarse dictionary Phi U D_low; problem (P_high)
 *     is OMP on y restricted to the columns f(Omega_low) of Phi D_high, the
 *     non-overlapping child blocks of Section III-B.  More than two scales
 *     chain the rule down the tree of Fig. 2 (each scale searches only the
 *     children of the previous scale's support).
 *
 * Readings of the paper used here (every one is listed in the design notes):
 *   - the child map is 0-based: children of coarse atom p are p*Q .. p*Q+Q-1;
 *   - the proxy divides |<a_i, r>| by ||a_i|| ("closest in angle"), which is
 *     the printed |<d_i, r>| when atoms have unit norm and Phi = I;
 *   - ties go to the lowest atom index; atoms already in the support, and
 *     atoms whose effective column is zero, are never picked;
 *   - the loop runs K times unless the candidates run out or the picked atom
 *     is numerically dependent on the support
 *     (||(I - P_Omega) a_k||^2 <= 1e-10 ||a_k||^2), in which case it stops;
 *   - every finer scale restarts from r = y and discards coarse coefficients;
 *   - U replicates a coarse value over its block (nearest neighbour), so the
 *     effective column at scale s is Phi applied to D_s[map_s(j), t];
 *   - Phi is the identity, a dense M x N matrix, or diag(mask) per patch.
 *
 * The projection re-solves the least-squares problem from scratch at every
 * step with Householder QR (Golub & Van Loan, Alg. 5.2.1 / 5.3.2), which is a
 * different route from the GPU's incremental Cholesky on purpose.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_SCALES 4
#define OR_DEP_TOL 1e-10

enum { OR_PHI_IDENTITY = 0, OR_PHI_DENSE = 1, OR_PHI_MASK = 2 };

/* Mirrors nothing in the product headers: the oracle's own model record. */
typedef struct {
    int32_t n_scales;
    int32_t dim[OR_MAX_SCALES];        /* N_s */
    int32_t atoms[OR_MAX_SCALES];      /* T_s */
    const double *dict[OR_MAX_SCALES]; /* column-major N_s x T_s */
    const int32_t *up_map[OR_MAX_SCALES]; /* s < S-1: length N_{s+1}, values in [0, N_s) */
    int32_t phi_kind;
    int32_t m;                         /* rows of Phi (= N for identity / mask) */
    const double *phi;                 /* row-major M x N for OR_PHI_DENSE, n_phases of them */
    int32_t n_phases;                  /* dense operators to choose from per patch (0 or 1: one) */
} oracle_model;

/* ---------------------------------------------------------------------- */
/* Least squares by Householder QR.                                        */
/* a: column-major m x n (copied), b: length m (copied).                   */
/* On return: beta (length n), and rdiag_last = |R[n-1][n-1]|, the length  */
/* of the part of the last column orthogonal to the span of the others.    */
/* ---------------------------------------------------------------------- */
static void householder_lstsq(const double *a, const double *b, int m, int n,
                              double *beta, double *rdiag_last, double *work)
{
    double *w = work;              /* m x n */
    double *c = work + (size_t)m * n; /* m */
    double *v = c + m;             /* m */
    memcpy(w, a, sizeof(double) * (size_t)m * n);
    memcpy(c, b, sizeof(double) * (size_t)m);
    for (int j = 0; j < n; ++j) {
        double *col = w + (size_t)j * m;
        double norm2 = 0.0;
        for (int i = j; i < m; ++i) norm2 += col[i] * col[i];
        double norm = sqrt(norm2);
        if (norm == 0.0) continue; /* zero column below the diagonal: R_jj = 0 */
        double alpha = col[j] > 0 ? -norm : norm;
        /* v = x - alpha e1, normalised */
        for (int i = j; i < m; ++i) v[i] = col[i];
        v[j] -= alpha;
        double vnorm2 = 0.0;
        for (int i = j; i < m; ++i) vnorm2 += v[i] * v[i];
        if (vnorm2 == 0.0) continue;
        double inv = 1.0 / sqrt(vnorm2);
        for (int i = j; i < m; ++i) v[i] *= inv;
        /* apply H = I - 2 v v^T to columns j..n-1 and to c */
        for (int k = j; k < n; ++k) {
            double *ck = w + (size_t)k * m;
            double dot = 0.0;
            for (int i = j; i < m; ++i) dot += v[i] * ck[i];
            for (int i = j; i < m; ++i) ck[i] -= 2.0 * dot * v[i];
        }
        double dot = 0.0;
        for (int i = j; i < m; ++i) dot += v[i] * c[i];
        for (int i = j; i < m; ++i) c[i] -= 2.0 * dot * v[i];
    }
    /* back substitution R beta = c[0..n-1] */
    for (int j = n - 1; j >= 0; --j) {
        double s = c[j];
        for (int k = j + 1; k < n; ++k) s -= w[(size_t)k * m + j] * beta[k];
        double rjj = w[(size_t)j * m + j];
        beta[j] = rjj != 0.0 ? s / rjj : 0.0;
    }
    *rdiag_last = n > 0 ? fabs(w[(size_t)(n - 1) * m + (n - 1)]) : 0.0;
}

/* ---------------------------------------------------------------------- */
/* Algorithm 1 on an explicit effective dictionary A (column-major M x T), */
/* searching only the candidate atoms cand[0..nc-1] (ascending indices).   */
/* ---------------------------------------------------------------------- */
typedef struct {
    int *support;      /* out, length kmax: selected atom indices in order */
    double *coef;      /* out, length kmax */
    int k_used;        /* out */
    const int *forced; /* in, length kmax or NULL; entries < 0 mean "free" */
    double *trace;     /* out, kmax x 4 or NULL: best, runner-up, picked score, step-1 max */
} omp_io;

static void omp_restricted(const double *A, int M, const int *cand, int nc,
                           const double *y, int K, omp_io *io, double *scratch)
{
    double *nu = scratch;               /* T-sized by candidate slot: nc */
    double *r = nu + nc;                /* M */
    double *asub = r + M;               /* M x K */
    double *work = asub + (size_t)M * K; /* (M x K) + 2M */
    double *beta = work + (size_t)M * K + 2 * (size_t)M; /* K */
    char *chosen = (char *)(beta + K);  /* nc */
    memset(chosen, 0, (size_t)nc);
    for (int c = 0; c < nc; ++c) {
        const double *a = A + (size_t)cand[c] * M;
        double s = 0.0;
        for (int i = 0; i < M; ++i) s += a[i] * a[i];
        nu[c] = sqrt(s);
    }
    memcpy(r, y, sizeof(double) * (size_t)M);
    int n = 0;
    double first_max = 0.0;
    for (int it = 0; it < K; ++it) {
        /* Proxy: score every remaining candidate against the residue. */
        int best = -1, second = -1;
        double bs = -1.0, ss = -1.0;
        for (int c = 0; c < nc; ++c) {
            if (chosen[c] || nu[c] == 0.0) continue;
            const double *a = A + (size_t)cand[c] * M;
            double dot = 0.0;
            for (int i = 0; i < M; ++i) dot += a[i] * r[i];
            double score = fabs(dot) / nu[c];
            if (score > bs) { ss = bs; second = best; bs = score; best = c; }
            else if (score > ss) { ss = score; second = c; }
        }
        (void)second;
        if (best < 0) break; /* candidates exhausted */
        if (it == 0) first_max = bs;
        int pick = best;
        double picked_score = bs;
        if (io->forced && io->forced[it] >= 0) {
            int want = io->forced[it];
            pick = -1;
            for (int c = 0; c < nc; ++c)
                if (cand[c] == want && !chosen[c] && nu[c] != 0.0) pick = c;
            if (pick < 0) break; /* forced atom not available: stop here */
            const double *a = A + (size_t)cand[pick] * M;
            double dot = 0.0;
            for (int i = 0; i < M; ++i) dot += a[i] * r[i];
            picked_score = fabs(dot) / nu[pick];
        }
        if (io->trace) {
            io->trace[it * 4 + 0] = bs;
            io->trace[it * 4 + 1] = ss;
            io->trace[it * 4 + 2] = picked_score;
            io->trace[it * 4 + 3] = first_max;
        }
        /* M independent atoms already span the measurement space, so any
         * further atom is dependent on them. */
        if (n >= M) break;
        /* Support merge (tentative) and projection. */
        memcpy(asub + (size_t)n * M, A + (size_t)cand[pick] * M, sizeof(double) * (size_t)M);
        double rlast = 0.0;
        householder_lstsq(asub, y, M, n + 1, beta, &rlast, work);
        if (rlast * rlast <= OR_DEP_TOL * nu[pick] * nu[pick]) break; /* dependent atom */
        chosen[pick] = 1;
        io->support[n] = cand[pick];
        ++n;
        for (int j = 0; j < n; ++j) io->coef[j] = beta[j];
        /* Residue. */
        for (int i = 0; i < M; ++i) {
            double s = y[i];
            for (int j = 0; j < n; ++j) s -= asub[(size_t)j * M + i] * beta[j];
            r[i] = s;
        }
    }
    io->k_used = n;
}

/* Effective dictionary at scale s for one patch: column t is
 * Phi applied to the upsampled atom u_j = D_s[map_s(j), t]. */
static void effective_dict(const oracle_model *md, int s, const int64_t *map_s,
                           const uint8_t *mask, const double *phi, double *A)
{
    const int N = md->dim[md->n_scales - 1];
    const int Ns = md->dim[s];
    const int T = md->atoms[s];
    const int M = md->m;
    const double *D = md->dict[s];
    for (int t = 0; t < T; ++t) {
        const double *d = D + (size_t)t * Ns;
        double *a = A + (size_t)t * M;
        if (md->phi_kind == OR_PHI_DENSE) {
            for (int i = 0; i < M; ++i) {
                double acc = 0.0;
                for (int j = 0; j < N; ++j) acc += phi[(size_t)i * N + j] * d[map_s[j]];
                a[i] = acc;
            }
        } else {
            for (int j = 0; j < N; ++j) {
                double u = d[map_s[j]];
                a[j] = (md->phi_kind == OR_PHI_MASK && !mask[j]) ? 0.0 : u;
            }
        }
    }
}

static void compose_maps(const oracle_model *md, int64_t **maps)
{
    const int S = md->n_scales;
    const int N = md->dim[S - 1];
    for (int j = 0; j < N; ++j) maps[S - 1][j] = j;
    for (int s = S - 2; s >= 0; --s)
        for (int j = 0; j < N; ++j) maps[s][j] = md->up_map[s][maps[s + 1][j]];
}

/*
 * Batched entry point.
 *   full != 0 : Algorithm 1 on the finest scale with every atom a candidate.
 *   full == 0 : zero-tree OMP through all scales.
 *   y        : B x M;  mask: B x N (OR_PHI_MASK only)
 *   k_scale  : K per scale (length S); k_fine (length B, may be NULL)
 *              overrides the finest scale's K per patch.
 *   forced   : B x S x kstride (or NULL), -1 = free step.
 *   supports : B x S x kstride out (-1 padded), coefs: B x S x kstride out,
 *   k_used   : B x S out, xhat: B x N out (may be NULL),
 *   trace    : B x S x kstride x 4 out (may be NULL).
 *   phase    : B (dense operators, n_phases > 1): which operator each
 *              patch is measured with; NULL means operator 0.
 * Returns 0, or -1 on a shape error.
 */
int oracle_omp(const oracle_model *md, int64_t B, const double *y, const uint8_t *mask,
               const int32_t *k_scale, const int32_t *k_fine, int32_t full,
               const int32_t *forced, int32_t kstride, int32_t *supports, double *coefs,
               int32_t *k_used, double *xhat, double *trace, int32_t n_threads,
               const int32_t *phase)
{
    const int S = md->n_scales;
    if (S < 1 || S > OR_MAX_SCALES) return -1;
    const int N = md->dim[S - 1];
    const int M = md->m;
    for (int s = 1; s < S; ++s)
        if (md->atoms[s] % md->atoms[s - 1] != 0) return -1;
    if (md->phi_kind != OR_PHI_DENSE && M != N) return -1;
    const int P = md->n_phases > 1 ? md->n_phases : 1;
    if (P > 1 && md->phi_kind != OR_PHI_DENSE) return -1;
    if (phase)
        for (int64_t b = 0; b < B; ++b) if (phase[b] < 0 || phase[b] >= P) return -1;
    int Tmax = 0, Kmax = 0;
    for (int s = 0; s < S; ++s) if (md->atoms[s] > Tmax) Tmax = md->atoms[s];
    for (int s = 0; s < S; ++s) if (k_scale[s] > Kmax) Kmax = k_scale[s];
    if (k_fine)
        for (int64_t b = 0; b < B; ++b) if (k_fine[b] > Kmax) Kmax = k_fine[b];
    if (Kmax > kstride) return -1;

    int64_t *maps[OR_MAX_SCALES];
    for (int s = 0; s < S; ++s) maps[s] = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    compose_maps(md, maps);

    /* Shared effective dictionaries when they do not depend on the patch
     * (one per operator when there are several). */
    double *shared[OR_MAX_SCALES] = {0};
    if (md->phi_kind != OR_PHI_MASK) {
        for (int s = 0; s < S; ++s) {
            const size_t one = (size_t)M * md->atoms[s];
            shared[s] = (double *)malloc(sizeof(double) * one * P);
            for (int p = 0; p < P; ++p)
                effective_dict(md, s, maps[s], NULL, md->phi ? md->phi + (size_t)p * M * N : NULL,
                               shared[s] + one * p);
        }
    }

#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
#endif
    {
        size_t kk = (size_t)(Kmax > 0 ? Kmax : 1);
        double *Aown = NULL;
        if (md->phi_kind == OR_PHI_MASK) Aown = (double *)malloc(sizeof(double) * (size_t)M * Tmax);
        int *cand = (int *)malloc(sizeof(int) * (size_t)Tmax);
        size_t scratch_n = (size_t)Tmax + M + (size_t)M * kk + (size_t)M * kk + 2 * (size_t)M + kk + (size_t)Tmax;
        double *scratch = (double *)malloc(sizeof(double) * scratch_n);
        int *prev = (int *)malloc(sizeof(int) * kk);
        int *sorted = (int *)malloc(sizeof(int) * kk);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t b = 0; b < B; ++b) {
            const double *yb = y + (size_t)b * M;
            const uint8_t *mb = mask ? mask + (size_t)b * N : NULL;
            int nprev = 0;
            int s0 = full ? S - 1 : 0;
            for (int s = 0; s < S; ++s) {
                k_used[b * S + s] = 0;
                for (int k = 0; k < kstride; ++k) {
                    supports[((size_t)b * S + s) * kstride + k] = -1;
                    coefs[((size_t)b * S + s) * kstride + k] = 0.0;
                }
            }
            for (int s = s0; s < S; ++s) {
                const double *A;
                if (md->phi_kind == OR_PHI_MASK) {
                    effective_dict(md, s, maps[s], mb, NULL, Aown);
                    A = Aown;
                } else {
                    A = shared[s] + (size_t)M * md->atoms[s] * (size_t)(phase ? phase[b] : 0);
                }
                int nc = 0;
                if (s == s0) {
                    for (int t = 0; t < md->atoms[s]; ++t) cand[nc++] = t;
                } else {
                    /* f(Omega): the union of the child blocks, ascending. */
                    int Q = md->atoms[s] / md->atoms[s - 1];
                    int np = nprev;
                    for (int i = 0; i < np; ++i) sorted[i] = prev[i];
                    for (int i = 1; i < np; ++i)
                        for (int j = i; j > 0 && sorted[j - 1] > sorted[j]; --j) {
                            int t = sorted[j]; sorted[j] = sorted[j - 1]; sorted[j - 1] = t;
                        }
                    for (int i = 0; i < np; ++i)
                        for (int q = 0; q < Q; ++q) cand[nc++] = sorted[i] * Q + q;
                }
                int K = k_scale[s];
                if (s == S - 1 && k_fine) K = k_fine[b];
                if (K > nc) K = nc;
                if (K < 0) K = 0;
                omp_io io;
                io.support = supports + ((size_t)b * S + s) * kstride;
                io.coef = coefs + ((size_t)b * S + s) * kstride;
                io.forced = forced ? forced + ((size_t)b * S + s) * kstride : NULL;
                io.trace = trace ? trace + (((size_t)b * S + s) * kstride) * 4 : NULL;
                io.k_used = 0;
                omp_restricted(A, M, cand, nc, yb, K, &io, scratch);
                k_used[b * S + s] = io.k_used;
                nprev = io.k_used;
                for (int i = 0; i < nprev; ++i) prev[i] = io.support[i];
            }
            if (xhat) {
                const double *Df = md->dict[S - 1];
                const int32_t *sup = supports + ((size_t)b * S + (S - 1)) * kstride;
                const double *cf = coefs + ((size_t)b * S + (S - 1)) * kstride;
                double *xb = xhat + (size_t)b * N;
                for (int j = 0; j < N; ++j) xb[j] = 0.0;
                for (int k = 0; k < k_used[b * S + S - 1]; ++k)
                    for (int j = 0; j < N; ++j) xb[j] += Df[(size_t)sup[k] * N + j] * cf[k];
            }
        }
        free(Aown); free(cand); free(scratch); free(prev); free(sorted);
    }
    for (int s = 0; s < S; ++s) { free(maps[s]); free(shared[s]); }
    return 0;
}

/* Threads an OpenMP region would use (for reporting). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

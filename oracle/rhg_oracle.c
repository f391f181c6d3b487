/*
 * rhg_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle for
 * threshold random hyperbolic graphs (von Looz, Oezdayi, Laue, Meyerhenke,
 * "Generating massive complex networks with hyperbolic geometry faster in
 * practice", HPEC 2016).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) includes, links or calls this file; only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark do.  It shares no
 * code, header, table or constant with the GPU path.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 *        -pthread rhg_oracle.c -lm
 * (no FMA contraction, no fast-math: every floating-point operation below is
 * one IEEE-754 binary64 round-to-nearest-even operation).
 *
 * Contents, each with the passage it follows:
 *   orc_kbar_approx / orc_target_radius  -- getTargetRadius (Sec. III-B,
 *        the average-degree approximation with zeta = 1, binary search on R).
 *   orc_boundaries                       -- radial slab boundaries, geometric
 *        widths with ratio p (Sec. III-A, Eq. 4).
 *   orc_splitmix64 / orc_sample          -- point distribution: angle uniform,
 *        radius with density alpha sinh(alpha r)/(cosh(alpha R)-1) (Sec. II,
 *        Eq. 1; Algorithm 1 sampling lines).  Random bits come from SplitMix64
 *        (Steele, Lea, Flood, OOPSLA 2014), written from its published
 *        definition.
 *   orc_table                            -- per-point FP64 values the
 *        distance test reads (exp(r), exp(-r), sinh r, sin(theta/2),
 *        cos(theta/2)), sinh r taken as (exp(r) - exp(-r)) / 2 of the first
 *        two.
 *   orc_coshdist / orc_is_edge           -- hyperbolic law of cosines (Sec. II,
 *        Eq. 3) against cosh R, evaluated in the cancellation-free form
 *        cosh(r_u - r_v) + 2 sinh r_u sinh r_v sin^2(dtheta/2).
 *   orc_brute                            -- the plain definition: all pairs.
 *   orc_window / orc_band_sweep          -- Algorithm 1's band query: slabs,
 *        angle sort per slab, getMinMaxPhi bound (Sec. III-B inequality chain),
 *        binary search of the window, outward-only scan.
 *   orc_move                             -- one movement step of the dynamic
 *        model (Sec. III-C: rotation, Algorithm 2's radial step, reflection
 *        at 0 and R), in the reading under which Theorem 1 holds (below).
 *   orc_pair_uniform / orc_fd_prob / orc_soft_brute / orc_soft_band_sweep
 *                                        -- the general model at temperature
 *        T > 0 (Sec. II, Eq. 2): each pair an edge with probability
 *        1/(exp((x - R)/(2T)) + 1) of its distance x, decided by one uniform
 *        per unordered pair (a reading: the paper gives no algorithm for
 *        T > 0); all pairs, and the band sweep with the radius enlarged to
 *        where that probability falls below the smallest uniform.
 *
 * Readings where the paper is silent or ambiguous (all listed in the design
 * notes of the repository): strict "< R"; half-open slabs with r = R in the
 * last slab; ceil(log2 n) slabs; (zeta/alpha)^2 in the degree formula; the
 * decreasing branch of that formula for the binary search; same-slab pairs
 * kept once by original index; the cancellation-free evaluation order above.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_TWO_PI (2.0 * 3.14159265358979323846) /* fl(2*pi): the angle period used by the sampler */

/* Domain of the disk radius.  Eq. 3 is evaluated below as
 * cosh(r_u - r_v) + 2 sinh r_u sinh r_v sin^2(dtheta/2); every product in it
 * must be finite for all pairs in the disk, or two coincident points on the
 * rim (sin = 0) would meet inf * 0 = NaN and be declared non-adjacent.  The
 * largest product is 2 sinh^2 R ~ e^{2R}/2, finite while 2R < ln(2 DBL_MAX)
 * = 710.48.  Radii up to 354 are accepted (a factor e^{2.4} below overflow);
 * beyond, the entry points return ORC_EDOMAIN. */
#define ORC_R_MAX 354.0
#define ORC_EDOMAIN (-2)

/* ------------------------------------------------------------------------- */
/* getTargetRadius (Sec. III-B).                                              */
/* ------------------------------------------------------------------------- */

/* Approximate expected average degree for n points, dispersion alpha, disk
 * radius R, with zeta = 1 and xi = (alpha/zeta)/(alpha/zeta - 1/2).  The
 * garbled "(zeta/alpha)^2" term is read as the square of zeta/alpha. */
double orc_kbar_approx(double n, double alpha, double R) {
    const double zeta = 1.0;
    double xi = (alpha / zeta) / (alpha / zeta - 0.5);
    double pre = (2.0 / ORC_PI) * xi * xi * n;
    double za = zeta / alpha;
    double first = pre * exp(-zeta * R / 2.0);
    double inner = alpha * (R / 2.0) * ((ORC_PI / 4.0) * za * za - (ORC_PI - 1.0) * za + (ORC_PI - 2.0)) - 1.0;
    double second = pre * (exp(-alpha * R) * inner);
    return first + second;
}

/* Binary search for R on the decreasing branch of orc_kbar_approx (the
 * function is 0 at R = 0, rises to a peak, then decays like e^{-R/2}).
 * Returns 0 on success, -1 if the target is not reachable (alpha <= 1/2,
 * non-positive target, or target above the peak). */
int orc_target_radius(double n, double alpha, double kbar, double *R_out) {
    if (!(n >= 2.0) || !(alpha > 0.5) || !(kbar > 0.0) || !isfinite(n) || !isfinite(alpha) || !isfinite(kbar))
        return -1;
    double xi = alpha / (alpha - 0.5);
    double rmax = 2.0 * log(n * xi * xi + 1.0) + 60.0;
    /* scan a fine grid from the right for the rightmost grid point whose
     * value reaches the target: the root lies between it and its right
     * neighbour, on the decreasing branch */
    const int steps = 200000;
    double h = rmax / steps;
    int found = -1;
    for (int i = steps; i >= 0; --i) {
        if (orc_kbar_approx(n, alpha, i * h) >= kbar) { found = i; break; }
    }
    if (found < 0 || found == steps) return -1;
    double lo = found * h, hi = (found + 1) * h; /* f(lo) >= kbar > f(hi) */
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (orc_kbar_approx(n, alpha, mid) >= kbar) lo = mid; else hi = mid;
    }
    *R_out = 0.5 * (lo + hi);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Radial boundaries (Sec. III-A, Eq. 4): c_0 = 0, c_B = R,                   */
/* c_{i+1} - c_i = p (c_i - c_{i-1}), c_1 = (1-p) R / (1 - p^B).              */
/* ------------------------------------------------------------------------- */
int orc_default_bands(uint64_t n) {
    int b = 0;
    while (b < 63 && ((uint64_t)1 << b) < n) ++b; /* ceil(log2 n) */
    return b < 1 ? 1 : b;
}

void orc_boundaries(double R, int B, double p, double *c) {
    double c1 = (1.0 - p) * R / (1.0 - pow(p, (double)B));
    c[0] = 0.0;
    double width = c1;
    for (int i = 1; i < B; ++i) {
        c[i] = c[i - 1] + width;
        width *= p;
    }
    c[B] = R;
}

/* Slab of radius r: the i with c_i <= r < c_{i+1}; r = R goes to the last. */
static int orc_band_of(double r, const double *c, int B) {
    int b = 0;
    while (b + 1 < B && c[b + 1] <= r) ++b;
    return b;
}

int orc_band_of_radius(double r, const double *c, int B) { return orc_band_of(r, c, B); }

/* ------------------------------------------------------------------------- */
/* Random points (Sec. II Eq. 1, Algorithm 1 sampling lines).                 */
/* ------------------------------------------------------------------------- */

/* SplitMix64: state advances by the golden gamma, output is the state passed
 * through the two xor-shift-multiply rounds.  The k-th output (k >= 0) of the
 * generator seeded with s is mix(s + (k+1) * gamma). */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * UINT64_C(0x9E3779B97F4A7C15);
    z = (z ^ (z >> 30)) * UINT64_C(0xBF58476D1CE4E5B9);
    z = (z ^ (z >> 27)) * UINT64_C(0x94D049BB133111EB);
    return z ^ (z >> 31);
}

/* Uniform on [0,1) with 53 random bits. */
static double orc_unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* Point i takes outputs 2i (angle) and 2i+1 (radius).
 * angle: u * fl(2 pi), in [0, fl(2 pi)).
 * radius: inverse of F(r) = (cosh(alpha r) - 1)/(cosh(alpha R) - 1)
 *       = sinh^2(alpha r / 2) / sinh^2(alpha R / 2),
 *   i.e. r = 2 asinh( sqrt(u) sinh(alpha R / 2) ) / alpha, clamped to [0, R]. */
int orc_sample_range(uint64_t i0, uint64_t i1, double alpha, double R, uint64_t seed, double *theta, double *r) {
    if (!(R > 0.0 && R <= ORC_R_MAX) || !(alpha > 0.0) || !isfinite(alpha)) return ORC_EDOMAIN;
    double sR = sinh(alpha * R / 2.0);
    if (!isfinite(sR)) return ORC_EDOMAIN; /* the inverse CDF needs sinh(alpha R / 2) */
    for (uint64_t i = i0; i < i1; ++i) {
        double u1 = orc_unit(orc_splitmix64(seed, 2 * i));
        double u2 = orc_unit(orc_splitmix64(seed, 2 * i + 1));
        theta[i] = u1 * ORC_TWO_PI;
        double ri = 2.0 * asinh(sqrt(u2) * sR) / alpha;
        r[i] = ri > R ? R : ri;
    }
    return 0;
}

int orc_sample(uint64_t n, double alpha, double R, uint64_t seed, double *theta, double *r) {
    return orc_sample_range(0, n, alpha, R, seed, theta, r);
}

/* ------------------------------------------------------------------------- */
/* Per-point table for the distance test.  sinh r is taken as                 */
/* (e^r - e^-r) / 2 from the two exponentials of the table (one rounded       */
/* subtraction, an exact halving), so that the distance test needs only four  */
/* independent values per point.  For small r the subtraction cancels: the    */
/* error is then absolute, at most about 3 u cosh r, and the term it feeds,   */
/* 2 sinh r_u sinh r_v sin^2(dtheta/2), stays within a few u of cosh dist.    */
/* ------------------------------------------------------------------------- */
void orc_table(uint64_t n, const double *theta, const double *r,
               double *ep, double *em, double *sh, double *hs, double *hc) {
    for (uint64_t i = 0; i < n; ++i) {
        ep[i] = exp(r[i]);
        em[i] = exp(-r[i]);
        sh[i] = 0.5 * (ep[i] - em[i]);
        hs[i] = sin(theta[i] / 2.0);
        hc[i] = cos(theta[i] / 2.0);
    }
}

typedef struct {
    const double *ep, *em, *sh, *hs, *hc;
} orc_tab;

/* cosh dist(u,v) by the hyperbolic law of cosines (Eq. 3), rewritten with
 *   cosh a cosh b - sinh a sinh b cos D = cosh(a-b) + 2 sinh a sinh b sin^2(D/2)
 *   cosh(a-b) = (e^a e^-b + e^-a e^b)/2,
 *   sin((t_u - t_v)/2) = sin(t_u/2)cos(t_v/2) - cos(t_u/2)sin(t_v/2).
 * One rounding per operation, in exactly this order; the result is bitwise
 * symmetric in (u, v). */
static double orc_V(const orc_tab *t, int64_t u, int64_t v) {
    double t1 = t->ep[u] * t->em[v];
    double t2 = t->em[u] * t->ep[v];
    double a = 0.5 * (t1 + t2);
    double d = t->hs[u] * t->hc[v] - t->hc[u] * t->hs[v];
    double b = (t->sh[u] * t->sh[v]) * (d * d);
    return a + 2.0 * b;
}

double orc_coshdist(const double *ep, const double *em, const double *sh, const double *hs, const double *hc,
                    int64_t u, int64_t v) {
    orc_tab t = {ep, em, sh, hs, hc};
    return orc_V(&t, u, v);
}

/* Edge iff the distance is below R: strict comparison against K = cosh R. */
int orc_is_edge(const double *ep, const double *em, const double *sh, const double *hs, const double *hc,
                int64_t u, int64_t v, double K) {
    if (u == v) return 0;
    orc_tab t = {ep, em, sh, hs, hc};
    return orc_V(&t, u, v) < K;
}

/* ------------------------------------------------------------------------- */
/* Growable edge buffer.                                                      */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t *p;
    int64_t m, cap;
    int oom;
} orc_buf;

static void orc_push(orc_buf *b, int64_t u, int64_t v) {
    if (b->oom) return;
    if (b->m == b->cap) {
        int64_t nc = b->cap ? 2 * b->cap : 1024;
        int32_t *np = (int32_t *)realloc(b->p, (size_t)nc * 2 * sizeof(int32_t));
        if (!np) { b->oom = 1; return; }
        b->p = np;
        b->cap = nc;
    }
    int64_t lo = u < v ? u : v, hi = u < v ? v : u;
    b->p[2 * b->m] = (int32_t)lo;
    b->p[2 * b->m + 1] = (int32_t)hi;
    b->m++;
}

void orc_free(void *p) { free(p); }

/* ------------------------------------------------------------------------- */
/* Brute force: every pair i < j (the plain definition of the edge set).      */
/* Output sorted lexicographically by construction.                           */
/* ------------------------------------------------------------------------- */
/* K = cosh R with R in the accepted domain (0, ORC_R_MAX]. */
static int orc_K_in_domain(double K) { return K > 1.0 && K <= cosh(ORC_R_MAX); }

int64_t orc_brute(int64_t n, const double *ep, const double *em, const double *sh, const double *hs,
                  const double *hc, double K, int32_t **out) {
    *out = NULL;
    if (!orc_K_in_domain(K)) return ORC_EDOMAIN;
    orc_tab t = {ep, em, sh, hs, hc};
    orc_buf b = {0};
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            if (orc_V(&t, i, j) < K) orc_push(&b, i, j);
    if (b.oom) { free(b.p); *out = NULL; return -1; }
    *out = b.p;
    return b.m;
}

/* ------------------------------------------------------------------------- */
/* Brute force for selected rows: all neighbours w of each listed query q    */
/* (the plain definition restricted to pairs touching q).  Output pairs are */
/* (q, w) in query-list order then increasing w; threads split the queries. */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t n, nq;
    const int64_t *q;
    orc_tab tab;
    double K;
    volatile int64_t next;
    orc_buf *bufs;
} orc_rows_ctx;

static void *orc_rows_worker(void *arg) {
    orc_rows_ctx *X = (orc_rows_ctx *)arg;
    for (;;) {
        int64_t k = __sync_fetch_and_add(&X->next, 1);
        if (k >= X->nq) break;
        int64_t v = X->q[k];
        orc_buf *b = &X->bufs[k];
        for (int64_t w = 0; w < X->n; ++w) {
            if (w == v) continue;
            if (orc_V(&X->tab, v, w) < X->K) {
                /* store (v, w) unordered: the row's own view */
                if (b->m == b->cap) {
                    int64_t nc = b->cap ? 2 * b->cap : 256;
                    int32_t *np = (int32_t *)realloc(b->p, (size_t)nc * 2 * sizeof(int32_t));
                    if (!np) { b->oom = 1; break; }
                    b->p = np;
                    b->cap = nc;
                }
                b->p[2 * b->m] = (int32_t)v;
                b->p[2 * b->m + 1] = (int32_t)w;
                b->m++;
            }
        }
    }
    return NULL;
}

int64_t orc_brute_rows(int64_t n, const double *ep, const double *em, const double *sh, const double *hs,
                       const double *hc, double K, const int64_t *queries, int64_t nq, int nthreads,
                       int32_t **out) {
    *out = NULL;
    if (!orc_K_in_domain(K)) return ORC_EDOMAIN;
    for (int64_t k = 0; k < nq; ++k)
        if (queries[k] < 0 || queries[k] >= n) return ORC_EDOMAIN;
    orc_rows_ctx X;
    memset(&X, 0, sizeof X);
    X.n = n; X.nq = nq; X.q = queries; X.K = K; X.next = 0;
    X.tab.ep = ep; X.tab.em = em; X.tab.sh = sh; X.tab.hs = hs; X.tab.hc = hc;
    X.bufs = (orc_buf *)calloc((size_t)(nq > 0 ? nq : 1), sizeof(orc_buf));
    if (!X.bufs) return -1;
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0;
    if (th) {
        for (int t = 0; t < nthreads; ++t)
            if (pthread_create(&th[t], NULL, orc_rows_worker, &X) == 0) ++started;
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
        free(th);
    }
    if (started == 0) orc_rows_worker(&X);
    int64_t m = 0;
    int oom = 0;
    for (int64_t k = 0; k < nq; ++k) { m += X.bufs[k].m; oom |= X.bufs[k].oom; }
    int32_t *all = oom ? NULL : (int32_t *)malloc((size_t)(m > 0 ? m : 1) * 2 * sizeof(int32_t));
    if (all) {
        int64_t at = 0;
        for (int64_t k = 0; k < nq; ++k) {
            if (X.bufs[k].m) memcpy(all + 2 * at, X.bufs[k].p, (size_t)X.bufs[k].m * 2 * sizeof(int32_t));
            at += X.bufs[k].m;
        }
    }
    for (int64_t k = 0; k < nq; ++k) free(X.bufs[k].p);
    free(X.bufs);
    if (!all) return -1;
    *out = all;
    return m;
}

/* ------------------------------------------------------------------------- */
/* getMinMaxPhi (Sec. III-B).  For query radius rv and slab inner boundary c, */
/* every neighbour w of v in the slab satisfies                               */
/*   cos|phi_w - phi_v| >= (cosh rv cosh c - cosh R) / (sinh rv sinh c).      */
/* Using 1 - cos x = 2 sin^2(x/2) and cosh a cosh b - sinh a sinh b =         */
/* cosh(a-b), the same bound reads                                            */
/*   sin^2(|phi_w - phi_v|/2) <= (cosh R - cosh(rv - c)) / (2 sinh rv sinh c) */
/* which has no cancellation for small windows.  Returns 1 if the whole slab  */
/* must be scanned, else 0 and the (widened) half-width in *delta.            */
/* Widening: the threshold is raised by a relative 1e-9 and the angle by a    */
/* relative 1e-9 plus an absolute 1e-13, which covers the rounding of the     */
/* table values, of the distance test, and of this computation, so that      */
/* every pair the distance test accepts lies inside the window.               */
/* ------------------------------------------------------------------------- */
int orc_window(double rv, double c, double K, double *delta) {
    double den = 2.0 * sinh(rv) * sinh(c);
    if (!(den > 0.0)) return 1;
    double Kw = K * (1.0 + 1e-9);
    double s = (Kw - cosh(rv - c)) / den;
    if (s >= 1.0) return 1;
    if (s < 0.0) s = 0.0;
    double d = 2.0 * asin(sqrt(s));
    d = d * (1.0 + 1e-9) + 1e-13;
    if (d >= ORC_PI) return 1;
    *delta = d;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Band sweep (Algorithm 1).                                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    double theta;
    int64_t id;
} orc_pt;

static int orc_cmp_pt(const void *a, const void *b) {
    const orc_pt *x = (const orc_pt *)a, *y = (const orc_pt *)b;
    if (x->theta < y->theta) return -1;
    if (x->theta > y->theta) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* first index in sorted[lo,hi) with theta >= x */
static int64_t orc_lower(const orc_pt *s, int64_t lo, int64_t hi, double x) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (s[mid].theta < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}
/* first index in sorted[lo,hi) with theta > x */
static int64_t orc_upper(const orc_pt *s, int64_t lo, int64_t hi, double x) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (s[mid].theta <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

typedef struct {
    /* shared, read-only */
    int64_t n, q0, q1, block;
    const double *theta, *r;
    orc_tab tab;
    double K;
    int B;
    const double *c;
    const int *band;
    const orc_pt *sorted;    /* all points, grouped by slab, angle-sorted within */
    const int64_t *band_off; /* B+1 */
    /* work distribution */
    int64_t nblocks;
    volatile int64_t next;
    orc_buf *bufs;    /* one per block */
    uint64_t *cands;  /* one per block */
} orc_sweep_ctx;

static void orc_scan_range(orc_sweep_ctx *X, int64_t v, int j, int64_t a, int64_t e, orc_buf *b, uint64_t *cand) {
    for (int64_t k = a; k < e; ++k) {
        int64_t w = X->sorted[k].id;
        if (w == v) continue;
        if (j == X->band[v] && w < v) continue; /* same slab: kept once, by the smaller index */
        ++*cand;
        if (orc_V(&X->tab, v, w) < X->K) orc_push(b, v, w);
    }
}

static void *orc_sweep_worker(void *arg) {
    orc_sweep_ctx *X = (orc_sweep_ctx *)arg;
    for (;;) {
        int64_t blk = __sync_fetch_and_add(&X->next, 1);
        if (blk >= X->nblocks) break;
        orc_buf *b = &X->bufs[blk];
        uint64_t cand = 0;
        int64_t v0 = X->q0 + blk * X->block;
        int64_t v1 = v0 + X->block < X->q1 ? v0 + X->block : X->q1;
        for (int64_t v = v0; v < v1; ++v) {
            double tv = X->theta[v], rv = X->r[v];
            for (int j = X->band[v]; j < X->B; ++j) { /* outward only */
                int64_t bs = X->band_off[j], be = X->band_off[j + 1];
                if (be == bs) continue;
                double delta;
                int whole = (j == 0) ? 1 : orc_window(rv, X->c[j], X->K, &delta);
                if (whole) {
                    orc_scan_range(X, v, j, bs, be, b, &cand);
                    continue;
                }
                double lo = tv - delta, hi = tv + delta;
                if (lo < 0.0) {
                    /* [0, hi] and [lo + 2pi, 2pi) */
                    orc_scan_range(X, v, j, bs, orc_upper(X->sorted, bs, be, hi), b, &cand);
                    orc_scan_range(X, v, j, orc_lower(X->sorted, bs, be, lo + ORC_TWO_PI), be, b, &cand);
                } else if (hi > ORC_TWO_PI) {
                    /* [lo, 2pi) and [0, hi - 2pi] */
                    orc_scan_range(X, v, j, orc_lower(X->sorted, bs, be, lo), be, b, &cand);
                    orc_scan_range(X, v, j, bs, orc_upper(X->sorted, bs, be, hi - ORC_TWO_PI), b, &cand);
                } else {
                    orc_scan_range(X, v, j, orc_lower(X->sorted, bs, be, lo), orc_upper(X->sorted, bs, be, hi), b,
                                   &cand);
                }
            }
        }
        X->cands[blk] = cand;
    }
    return NULL;
}

/* Band sweep over queries v in [q0, q1) (all queries: q0 = 0, q1 = n).
 * Every point is inserted in its slab and the slabs are angle-sorted; only
 * the queries in [q0, q1) are processed (a contiguous index range of i.i.d.
 * points is a uniform sample, used for time-bounded CPU baselines).
 * The windows of a wrapped interval are split in two ranges.  Output edges
 * are (min, max) original indices, concatenated in query-block order (a
 * deterministic order); candidates_out receives the number of distance
 * tests.  Returns m, or -1 on allocation failure. */
int64_t orc_band_sweep(int64_t n, const double *theta, const double *r, const double *ep, const double *em,
                       const double *sh, const double *hs, const double *hc, double R, double K, int B, double p,
                       int nthreads, int64_t q0, int64_t q1, int32_t **out, uint64_t *candidates_out) {
    *out = NULL;
    if (B < 1 || n < 0 || q0 < 0 || q1 > n || q0 > q1) return -1;
    if (!(R > 0.0 && R <= ORC_R_MAX) || !orc_K_in_domain(K)) return ORC_EDOMAIN;
    double *c = (double *)malloc((size_t)(B + 1) * sizeof(double));
    int *band = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    int64_t *band_off = (int64_t *)calloc((size_t)B + 1, sizeof(int64_t));
    orc_pt *sorted = (orc_pt *)malloc((size_t)(n > 0 ? n : 1) * sizeof(orc_pt));
    int64_t *fill = (int64_t *)calloc((size_t)B + 1, sizeof(int64_t));
    if (!c || !band || !band_off || !sorted || !fill) {
        free(c); free(band); free(band_off); free(sorted); free(fill);
        return -1;
    }
    orc_boundaries(R, B, p, c);
    for (int64_t v = 0; v < n; ++v) {
        band[v] = orc_band_of(r[v], c, B);
        band_off[band[v] + 1]++;
    }
    for (int j = 0; j < B; ++j) band_off[j + 1] += band_off[j];
    for (int64_t v = 0; v < n; ++v) {
        int64_t k = band_off[band[v]] + fill[band[v]]++;
        sorted[k].theta = theta[v];
        sorted[k].id = v;
    }
    for (int j = 0; j < B; ++j)
        qsort(sorted + band_off[j], (size_t)(band_off[j + 1] - band_off[j]), sizeof(orc_pt), orc_cmp_pt);

    orc_sweep_ctx X;
    memset(&X, 0, sizeof X);
    X.n = n; X.q0 = q0; X.q1 = q1; X.block = 2048;
    X.theta = theta; X.r = r;
    X.tab.ep = ep; X.tab.em = em; X.tab.sh = sh; X.tab.hs = hs; X.tab.hc = hc;
    X.K = K; X.B = B; X.c = c; X.band = band; X.sorted = sorted; X.band_off = band_off;
    X.nblocks = (q1 - q0 + X.block - 1) / X.block;
    X.next = 0;
    X.bufs = (orc_buf *)calloc((size_t)(X.nblocks > 0 ? X.nblocks : 1), sizeof(orc_buf));
    X.cands = (uint64_t *)calloc((size_t)(X.nblocks > 0 ? X.nblocks : 1), sizeof(uint64_t));
    int64_t m = -1;
    if (X.bufs && X.cands) {
        if (nthreads < 1) nthreads = 1;
        pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
        int started = 0;
        if (th) {
            for (int t = 0; t < nthreads; ++t)
                if (pthread_create(&th[t], NULL, orc_sweep_worker, &X) == 0) ++started;
            for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
            free(th);
        }
        if (started == 0) orc_sweep_worker(&X);
        int oom = 0;
        m = 0;
        uint64_t cand = 0;
        for (int64_t k = 0; k < X.nblocks; ++k) {
            m += X.bufs[k].m;
            cand += X.cands[k];
            oom |= X.bufs[k].oom;
        }
        int32_t *all = oom ? NULL : (int32_t *)malloc((size_t)(m > 0 ? m : 1) * 2 * sizeof(int32_t));
        if (!all) {
            m = -1;
        } else {
            int64_t at = 0;
            for (int64_t k = 0; k < X.nblocks; ++k) {
                if (X.bufs[k].m) memcpy(all + 2 * at, X.bufs[k].p, (size_t)X.bufs[k].m * 2 * sizeof(int32_t));
                at += X.bufs[k].m;
            }
            *out = all;
        }
        if (candidates_out) *candidates_out = cand;
        for (int64_t k = 0; k < X.nblocks; ++k) free(X.bufs[k].p);
    }
    free(X.bufs); free(X.cands);
    free(c); free(band); free(band_off); free(sorted); free(fill);
    return m;
}

/* ------------------------------------------------------------------------- */
/* Canonical order of an edge list: lexicographic (lo, hi).                   */
/* ------------------------------------------------------------------------- */
static int orc_cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

void orc_sort_edges(int32_t *pairs, int64_t m) {
    uint64_t *k = (uint64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
    if (!k) return;
    for (int64_t i = 0; i < m; ++i) k[i] = ((uint64_t)(uint32_t)pairs[2 * i] << 32) | (uint32_t)pairs[2 * i + 1];
    qsort(k, (size_t)m, sizeof(uint64_t), orc_cmp_u64);
    for (int64_t i = 0; i < m; ++i) {
        pairs[2 * i] = (int32_t)(k[i] >> 32);
        pairs[2 * i + 1] = (int32_t)(k[i] & 0xffffffffu);
    }
    free(k);
}

/* ------------------------------------------------------------------------- */
/* Dynamic model: one movement step (Sec. III-C, Algorithm 2, Theorem 1).     */
/*                                                                            */
/* Rotation: theta' = (theta + tau_phi) mod 2 pi, into [0, fl(2 pi)).         */
/* Radial step: Algorithm 2 adds tau_r to a transform of r under which the    */
/* radius density of Eq. 1 is uniform and maps back.  Under the density       */
/* alpha sinh(alpha r) / (cosh(alpha R) - 1) that transform is                */
/* w = cosh(alpha r), uniform on [1, cosh(alpha R)] (the interval starting at */
/* 1 that the paper's figure of the movement shows); the printed sinh is not  */
/* uniform near the centre and would not preserve the density, as Theorem 1   */
/* states it does.  The step is taken in the equivalent variable               */
/*   s = (w - 1) / 2 = sinh^2(alpha r / 2),  uniform on [0, S], S = sinh^2(alpha R / 2),   */
/* by s + tau_r / 2, which keeps its precision near the centre.  A step that  */
/* leaves [0, S] is reflected at the end it crosses (mirror), as often as it  */
/* crosses one, and each reflection negates tau_r (the node bounces):         */
/*   y = s + tau_r / 2,  k = floor(y / S);                                    */
/*   s' = y - k S (k even) or (k + 1) S - y (k odd),  tau_r' = (-1)^k tau_r.  */
/* Then r' = 2 asinh(sqrt(s')) / alpha, clamped to [0, R].  Reflection maps    */
/* the uniform law on [0, S] to itself for each step size when both signs of  */
/* the step are equally likely (Theorem 1 then holds exactly at every step).  */
/* ------------------------------------------------------------------------- */
void orc_move(uint64_t n, double alpha, double R, double *theta, double *r, const double *tau_phi,
              double *tau_r) {
    const double hS = sinh(alpha * R / 2.0);
    const double S = hS * hS;
    for (uint64_t i = 0; i < n; ++i) {
        /* rotation */
        double t = theta[i] + tau_phi[i];
        t = t - ORC_TWO_PI * floor(t / ORC_TWO_PI);
        if (t >= ORC_TWO_PI) t = 0.0;
        if (t < 0.0) t = 0.0;
        theta[i] = t;
        /* radial step on s = sinh^2(alpha r / 2), reflected into [0, S]; a zero
         * step leaves the radius exactly as it is */
        if (tau_r[i] == 0.0) continue;
        const double h = sinh(alpha * r[i] / 2.0);
        const double y = h * h + tau_r[i] / 2.0;
        const double k = floor(y / S);
        const int odd = fmod(fabs(k), 2.0) == 1.0;
        double s2 = odd ? (k + 1.0) * S - y : y - k * S;
        if (s2 < 0.0) s2 = 0.0;
        if (s2 > S) s2 = S;
        if (odd) tau_r[i] = -tau_r[i];
        double r2 = 2.0 * asinh(sqrt(s2)) / alpha;
        r[i] = r2 > R ? R : r2;
    }
}


/* ------------------------------------------------------------------------- */
/* General model, temperature T > 0 (Sec. II, Eq. 2).                         */
/*                                                                            */
/* Eq. 2 gives pair {u, v} at distance x the edge probability                 */
/*   f(x) = 1 / (exp((x - R) / (2 T)) + 1).                                   */
/* The paper gives no algorithm for T > 0; the reading used here decides      */
/* each unordered pair {lo, hi} (lo < hi, original indices) once, with its    */
/* own uniform U in (0, 1]: edge iff U < f(x).  U comes from the points'      */
/* SplitMix64 generator (same seed) at output 2^62 + lo 2^31 + hi, far from   */
/* the outputs 0 .. 2n - 1 the points use (n < 2^31), mapped to               */
/* ((z >> 11) + 1) 2^-53.  x = acosh(V) with V the cosh distance of Eq. 3 as  */
/* evaluated above (x = 0 for V <= 1: rounding can put coincident points a    */
/* hair below 1), y = (x - R) / (2 T), f = 1 / (1 + exp(y)), all FP64.        */
/* ------------------------------------------------------------------------- */
double orc_pair_uniform(uint64_t seed, int64_t lo, int64_t hi) {
    uint64_t k = ((uint64_t)1 << 62) + ((uint64_t)lo << 31) + (uint64_t)hi;
    uint64_t z = orc_splitmix64(seed, k);
    return (double)((z >> 11) + 1) * (1.0 / 9007199254740992.0);
}

double orc_fd_prob(double V, double R, double T) {
    double x = V > 1.0 ? acosh(V) : 0.0;
    double y = (x - R) / (2.0 * T);
    return 1.0 / (1.0 + exp(y));
}

/* Relative width of the band around f within which two correct FP64
 * evaluations of f from the same V may fall on different sides of U: acosh
 * within 2 ulp on either side (4 ulp of x apart), scaled by 1/(2T) in y, plus
 * a few ulp for exp and the division; taken 4 times over. */
static double orc_tie_width(double V, double T) {
    double x = V > 1.0 ? acosh(V) : 1.0;
    if (x < 1.0) x = 1.0;
    double ulp = nextafter(x, INFINITY) - x;
    return 16.0 * ulp / (2.0 * T) + 0x1p-45;
}

static int orc_T_ok(double R, double T) {
    return T > 0.0 && T < 1.0 && isfinite(T) && R > 0.0 && R <= ORC_R_MAX;
}

int orc_soft_is_edge(const double *ep, const double *em, const double *sh, const double *hs, const double *hc,
                     int64_t u, int64_t v, double R, double T, uint64_t seed) {
    if (u == v) return 0;
    orc_tab t = {ep, em, sh, hs, hc};
    int64_t lo = u < v ? u : v, hi = u < v ? v : u;
    return orc_pair_uniform(seed, lo, hi) < orc_fd_prob(orc_V(&t, u, v), R, T);
}

/* Edge decision of one pair, and whether it is a near tie (U within the
 * rounding band of f). */
static int orc_soft_decide(const orc_tab *t, int64_t u, int64_t v, double R, double T, uint64_t seed, int *tie) {
    int64_t lo = u < v ? u : v, hi = u < v ? v : u;
    double V = orc_V(t, u, v);
    double U = orc_pair_uniform(seed, lo, hi);
    double f = orc_fd_prob(V, R, T);
    *tie = fabs(U - f) <= orc_tie_width(V, T) * f;
    return U < f;
}

/* All pairs i < j (the plain definition).  Near ties go to *ties (may be
 * NULL).  Returns m, ORC_EDOMAIN, or -1 on allocation failure. */
int64_t orc_soft_brute(int64_t n, const double *ep, const double *em, const double *sh, const double *hs,
                       const double *hc, double R, double T, uint64_t seed, int32_t **out, int32_t **ties,
                       int64_t *nties) {
    *out = NULL;
    if (ties) *ties = NULL;
    if (nties) *nties = 0;
    if (!orc_T_ok(R, T)) return ORC_EDOMAIN;
    orc_tab t = {ep, em, sh, hs, hc};
    orc_buf b = {0}, tb = {0};
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            int tie = 0;
            if (orc_soft_decide(&t, i, j, R, T, seed, &tie)) orc_push(&b, i, j);
            if (tie) orc_push(&tb, i, j);
        }
    if (b.oom || tb.oom) { free(b.p); free(tb.p); return -1; }
    *out = b.p;
    if (ties) *ties = tb.p; else free(tb.p);
    if (nties) *nties = tb.m;
    return b.m;
}

/* Band sweep of the general model: Algorithm 1's slabs, angle sort and
 * getMinMaxPhi windows, for the enlarged radius Rc = R + 80 T (beyond it
 * y > 40 and f < e^-40 < 2^-53 <= U: no pair there can be an edge), then the
 * decision above for every candidate.  Same-slab pairs once, by index.  As
 * orc_band_sweep, plus the near ties in *ties. */
typedef struct {
    int64_t n, block, nblocks;
    const double *theta, *r;
    orc_tab tab;
    double R, T, Kc;
    uint64_t seed;
    int B;
    const double *c;
    const int *band;
    const orc_pt *sorted;
    const int64_t *band_off;
    volatile int64_t next;
    orc_buf *bufs, *tbufs;
    uint64_t *cands;
} orc_soft_ctx;

static void orc_soft_range(orc_soft_ctx *X, int64_t v, int j, int64_t a, int64_t e, orc_buf *b, orc_buf *tb,
                           uint64_t *cand) {
    for (int64_t k = a; k < e; ++k) {
        int64_t w = X->sorted[k].id;
        if (w == v) continue;
        if (j == X->band[v] && w < v) continue;
        ++*cand;
        int tie = 0;
        if (orc_soft_decide(&X->tab, v, w, X->R, X->T, X->seed, &tie)) orc_push(b, v, w);
        if (tie) orc_push(tb, v, w);
    }
}

static void *orc_soft_worker(void *arg) {
    orc_soft_ctx *X = (orc_soft_ctx *)arg;
    for (;;) {
        int64_t blk = __sync_fetch_and_add(&X->next, 1);
        if (blk >= X->nblocks) break;
        orc_buf *b = &X->bufs[blk], *tb = &X->tbufs[blk];
        uint64_t cand = 0;
        int64_t v0 = blk * X->block, v1 = v0 + X->block < X->n ? v0 + X->block : X->n;
        for (int64_t v = v0; v < v1; ++v) {
            double tv = X->theta[v], rv = X->r[v];
            for (int j = X->band[v]; j < X->B; ++j) {
                int64_t bs = X->band_off[j], be = X->band_off[j + 1];
                if (be == bs) continue;
                double delta;
                int whole = (j == 0) ? 1 : orc_window(rv, X->c[j], X->Kc, &delta);
                if (whole) {
                    orc_soft_range(X, v, j, bs, be, b, tb, &cand);
                    continue;
                }
                double lo = tv - delta, hi = tv + delta;
                if (lo < 0.0) {
                    orc_soft_range(X, v, j, bs, orc_upper(X->sorted, bs, be, hi), b, tb, &cand);
                    orc_soft_range(X, v, j, orc_lower(X->sorted, bs, be, lo + ORC_TWO_PI), be, b, tb, &cand);
                } else if (hi > ORC_TWO_PI) {
                    orc_soft_range(X, v, j, orc_lower(X->sorted, bs, be, lo), be, b, tb, &cand);
                    orc_soft_range(X, v, j, bs, orc_upper(X->sorted, bs, be, hi - ORC_TWO_PI), b, tb, &cand);
                } else {
                    orc_soft_range(X, v, j, orc_lower(X->sorted, bs, be, lo), orc_upper(X->sorted, bs, be, hi), b,
                                   tb, &cand);
                }
            }
        }
        X->cands[blk] = cand;
    }
    return NULL;
}

static int32_t *orc_concat(orc_buf *bufs, int64_t nb, int64_t *m_out) {
    int64_t m = 0;
    for (int64_t k = 0; k < nb; ++k) {
        if (bufs[k].oom) return NULL;
        m += bufs[k].m;
    }
    int32_t *all = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * 2 * sizeof(int32_t));
    if (!all) return NULL;
    int64_t at = 0;
    for (int64_t k = 0; k < nb; ++k) {
        if (bufs[k].m) memcpy(all + 2 * at, bufs[k].p, (size_t)bufs[k].m * 2 * sizeof(int32_t));
        at += bufs[k].m;
    }
    *m_out = m;
    return all;
}

int64_t orc_soft_band_sweep(int64_t n, const double *theta, const double *r, const double *ep, const double *em,
                            const double *sh, const double *hs, const double *hc, double R, double T, uint64_t seed,
                            int B, double p, int nthreads, int32_t **out, int32_t **ties, int64_t *nties,
                            uint64_t *candidates_out) {
    *out = NULL;
    *ties = NULL;
    *nties = 0;
    if (B < 1 || n < 0) return -1;
    if (!orc_T_ok(R, T)) return ORC_EDOMAIN;
    double *c = (double *)malloc((size_t)(B + 1) * sizeof(double));
    int *band = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    int64_t *band_off = (int64_t *)calloc((size_t)B + 1, sizeof(int64_t));
    orc_pt *sorted = (orc_pt *)malloc((size_t)(n > 0 ? n : 1) * sizeof(orc_pt));
    int64_t *fill = (int64_t *)calloc((size_t)B + 1, sizeof(int64_t));
    if (!c || !band || !band_off || !sorted || !fill) {
        free(c); free(band); free(band_off); free(sorted); free(fill);
        return -1;
    }
    /* slabs of the disk of radius R (the points' disk); windows for Rc */
    orc_boundaries(R, B, p, c);
    for (int64_t v = 0; v < n; ++v) {
        band[v] = orc_band_of(r[v], c, B);
        band_off[band[v] + 1]++;
    }
    for (int j = 0; j < B; ++j) band_off[j + 1] += band_off[j];
    for (int64_t v = 0; v < n; ++v) {
        int64_t k = band_off[band[v]] + fill[band[v]]++;
        sorted[k].theta = theta[v];
        sorted[k].id = v;
    }
    for (int j = 0; j < B; ++j)
        qsort(sorted + band_off[j], (size_t)(band_off[j + 1] - band_off[j]), sizeof(orc_pt), orc_cmp_pt);
    orc_soft_ctx X;
    memset(&X, 0, sizeof X);
    X.n = n; X.block = 1024; X.nblocks = (n + X.block - 1) / X.block;
    X.theta = theta; X.r = r;
    X.tab.ep = ep; X.tab.em = em; X.tab.sh = sh; X.tab.hs = hs; X.tab.hc = hc;
    X.R = R; X.T = T; X.seed = seed; X.Kc = cosh(R + 80.0 * T);
    X.B = B; X.c = c; X.band = band; X.sorted = sorted; X.band_off = band_off;
    X.next = 0;
    int64_t nbk = X.nblocks > 0 ? X.nblocks : 1;
    X.bufs = (orc_buf *)calloc((size_t)nbk, sizeof(orc_buf));
    X.tbufs = (orc_buf *)calloc((size_t)nbk, sizeof(orc_buf));
    X.cands = (uint64_t *)calloc((size_t)nbk, sizeof(uint64_t));
    int64_t m = -1;
    if (X.bufs && X.tbufs && X.cands) {
        if (nthreads < 1) nthreads = 1;
        pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
        int started = 0;
        if (th) {
            for (int t = 0; t < nthreads; ++t)
                if (pthread_create(&th[t], NULL, orc_soft_worker, &X) == 0) ++started;
            for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
            free(th);
        }
        if (started == 0) orc_soft_worker(&X);
        int64_t mt = 0;
        int32_t *all = orc_concat(X.bufs, X.nblocks, &m);
        int32_t *tall = all ? orc_concat(X.tbufs, X.nblocks, &mt) : NULL;
        if (!all || !tall) {
            free(all); free(tall);
            m = -1;
        } else {
            *out = all;
            *ties = tall;
            *nties = mt;
            uint64_t cand = 0;
            for (int64_t k = 0; k < X.nblocks; ++k) cand += X.cands[k];
            if (candidates_out) *candidates_out = cand;
        }
        for (int64_t k = 0; k < X.nblocks; ++k) { free(X.bufs[k].p); free(X.tbufs[k].p); }
    }
    free(X.bufs); free(X.tbufs); free(X.cands);
    free(c); free(band); free(band_off); free(sorted); free(fill);
    return m;
}

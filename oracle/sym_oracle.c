/*
 * sym_oracle.c -- plain FP64 CPU oracle for the one-loop Symanzik improved gauge
 * action, its molecular-dynamics force and a leapfrog trajectory built on them.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this library. It shares no code, header, table or helper with
 * the GPU library, and the GPU library never calls it.
 *
 * Source: D. Li, "The Calculation of Force in Lattice QCD", arXiv:1808.02281, Sec. II
 * ("One-loop Symanzik improved action"). Everything here is written straight from the
 * definitions and the force algorithm of that section, in FP64, with no blocking,
 * fusion or sharing of partial products:
 *
 *   - loop set: eq. (18_3_27_30) -- per site 6 plaquettes (mu,nu,-mu,-nu) mu<nu,
 *     12 rectangles (mu,mu,nu,-mu,-mu,-nu) mu!=nu, 16 cube loops
 *     (mu,+-nu,+-rho,-mu,-+nu,-+rho) mu<nu<rho;
 *   - coefficients c_P: eq. (18_3_27_30) and alpha_s = -4 log(u0)/3.06839;
 *   - loop products P_n = U_{n1,d1}...U_{nL,dL}: eq. (18_6_6_3_0), with
 *     U_{n,-mu} = U^dagger_{n-mu,mu};
 *   - action S_G = beta/3 sum_n sum_P c_P [3 - Re tr P_n]: eq. (18_6_4_1);
 *   - force: (beta/6) i (U_{k,rho} t_{k,rho})_TA with the TA projection of
 *     eq. (18_6_6_11), where t_{k,rho} collects, with weight c_P, the derivative of
 *     Re tr P_n with respect to U_{k,rho} for every loop instance through the link
 *     (eq. 18_7_25_2). The whole field is built by scattering: each loop instance is
 *     walked once and deposits its staple into every link it contains. Single links
 *     are gathered by the rotation rules of the force algorithm after eq. (18_6_6_13)
 *     (staple from k+rho, reversed and daggered for d_l = -rho); the two formulations
 *     share only the loop walk and are checked against each other. This file returns
 *     G = (beta/6)(U t)_TA, the antihermitian matrix; the paper's Hermitian force is iG.
 *
 * Parity-relevant readings of the paper:
 *   - U_{n,mu} lives on the link (n, n+mu) (the paper's text has a typo there);
 *   - the factor i of the force sits outside the TA projection;
 *   - all four directions are periodic; mu = 0..3 is x,y,z,t; x runs fastest;
 *   - "log" is the natural logarithm.
 *
 * Layout: canonical array-of-structures, lexicographic. Link (site s, direction mu)
 * is the 3x3 complex matrix at U[(s*4 + mu)*9 + 3*row + col], with
 * s = ((t*Lz + z)*Ly + y)*Lx + x. Momenta use the same layout.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;
typedef struct { cplx a[3][3]; } mat3;

/* ---------------------------------------------------------------- 3x3 algebra */

static mat3 m_zero(void) { mat3 r; memset(&r, 0, sizeof r); return r; }

static mat3 m_unit(void) {
    mat3 r = m_zero();
    for (int i = 0; i < 3; ++i) r.a[i][i] = 1.0;
    return r;
}

static mat3 m_mul(mat3 x, mat3 y) {
    mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < 3; ++k) s += x.a[i][k] * y.a[k][j];
            r.a[i][j] = s;
        }
    return r;
}

static mat3 m_dag(mat3 x) {
    mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = conj(x.a[j][i]);
    return r;
}

static mat3 m_add_scaled(mat3 x, double c, mat3 y) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) x.a[i][j] += c * y.a[i][j];
    return x;
}

static mat3 m_scale(mat3 x, cplx c) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) x.a[i][j] *= c;
    return x;
}

static cplx m_trace(mat3 x) { return x.a[0][0] + x.a[1][1] + x.a[2][2]; }

/* eq. (18_6_6_11): B_TA = (B - B^dag)/2 - tr(B - B^dag)/6 * I */
static mat3 m_ta(mat3 b) {
    mat3 d = m_add_scaled(b, -1.0, m_dag(b));
    cplx tr = m_trace(d);
    mat3 r = m_scale(d, 0.5);
    for (int i = 0; i < 3; ++i) r.a[i][i] -= tr / 6.0;
    return r;
}

static double m_norm1(mat3 x) { /* max column sum of |x_ij| */
    double best = 0.0;
    for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int i = 0; i < 3; ++i) s += cabs(x.a[i][j]);
        if (s > best) best = s;
    }
    return best;
}

static mat3 m_load(const cplx *p) {
    mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = p[3 * i + j];
    return r;
}

static void m_store(cplx *p, mat3 x) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) p[3 * i + j] = x.a[i][j];
}

/* ------------------------------------------------------------------ geometry */

typedef struct { int L[4]; int64_t V; } lattice;

static lattice make_lattice(const int32_t L[4]) {
    lattice g;
    g.V = 1;
    for (int m = 0; m < 4; ++m) { g.L[m] = L[m]; g.V *= L[m]; }
    return g;
}

static void site_coords(const lattice *g, int64_t s, int x[4]) {
    for (int m = 0; m < 4; ++m) { x[m] = (int)(s % g->L[m]); s /= g->L[m]; }
}

static int64_t site_index(const lattice *g, const int x[4]) {
    int64_t s = 0;
    for (int m = 3; m >= 0; --m) s = s * g->L[m] + x[m];
    return s;
}

/* n + d-hat for a signed direction d in {+-1..+-4} (axis |d|-1), periodic. */
static int64_t step(const lattice *g, int64_t s, int d) {
    int x[4];
    site_coords(g, s, x);
    int m = abs(d) - 1;
    x[m] = (x[m] + (d > 0 ? 1 : g->L[m] - 1)) % g->L[m];
    return site_index(g, x);
}

/* U_{n,d}; for a negative direction U_{n,-mu} = U^dagger_{n-mu,mu} (Sec. II). */
static mat3 link(const lattice *g, const cplx *U, int64_t n, int d) {
    if (d > 0) return m_load(U + (n * 4 + (d - 1)) * 9);
    int64_t back = step(g, n, d); /* n - mu */
    return m_dag(m_load(U + (back * 4 + (-d - 1)) * 9));
}

/* ------------------------------------------------------------------ loop set */

enum { CLS_PLAQ = 0, CLS_RECT = 1, CLS_CUBE = 2 };

typedef struct { int len; int cls; int d[6]; } loop_t;

/* eq. (18_3_27_30): the 34 closed paths that begin and end at every site. */
static int build_loops(loop_t out[34]) {
    int n = 0;
    for (int mu = 1; mu <= 4; ++mu)
        for (int nu = mu + 1; nu <= 4; ++nu) {
            loop_t p = {4, CLS_PLAQ, {mu, nu, -mu, -nu, 0, 0}};
            out[n++] = p;
        }
    for (int mu = 1; mu <= 4; ++mu)
        for (int nu = 1; nu <= 4; ++nu) {
            if (nu == mu) continue;
            loop_t p = {6, CLS_RECT, {mu, mu, nu, -mu, -mu, -nu}};
            out[n++] = p;
        }
    for (int mu = 1; mu <= 4; ++mu)
        for (int nu = mu + 1; nu <= 4; ++nu)
            for (int rho = nu + 1; rho <= 4; ++rho)
                for (int s = -1; s <= 1; s += 2)
                    for (int t = -1; t <= 1; t += 2) {
                        loop_t p = {6, CLS_CUBE, {mu, s * nu, t * rho, -mu, -s * nu, -t * rho}};
                        out[n++] = p;
                    }
    return n;
}

/* P_n = U_{n1,d1} ... U_{nL,dL}, n1 = n, n_{i+1} = n_i + d_i (eq. 18_6_6_3_0). */
static mat3 loop_product(const lattice *g, const cplx *U, int64_t n, const loop_t *p) {
    mat3 r = m_unit();
    int64_t s = n;
    for (int i = 0; i < p->len; ++i) {
        r = m_mul(r, link(g, U, s, p->d[i]));
        s = step(g, s, p->d[i]);
    }
    return r;
}

/* ------------------------------------------------------------- coefficients */

/* c[0] plaquette, c[1] rectangle, c[2] cube (eq. 18_3_27_30 and the alpha_s formula). */
int orc_coeffs(double u0, double c[3], double *alpha_s) {
    if (!(u0 > 0.0) || !isfinite(u0)) return -1;
    double as = -4.0 * log(u0) / 3.06839;
    c[0] = 1.0;
    c[1] = -(1.0 + 0.4805 * as) / (20.0 * u0 * u0);
    c[2] = -2.0 * 0.03325 * as / (u0 * u0);
    if (alpha_s) *alpha_s = as;
    return 0;
}

int orc_loop_table(int32_t *len, int32_t *cls, int32_t *dirs /* 34*6 */) {
    loop_t lp[34];
    int n = build_loops(lp);
    for (int i = 0; i < n; ++i) {
        len[i] = lp[i].len;
        cls[i] = lp[i].cls;
        for (int j = 0; j < 6; ++j) dirs[6 * i + j] = lp[i].d[j];
    }
    return n;
}

/* ----------------------------------------------------------------- summation */

/* Neumaier compensated summation. */
typedef struct { double s, c; } ksum;
static void ks_add(ksum *k, double v) {
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static double ks_val(const ksum *k) { return k->s + k->c; }

/* -------------------------------------------------------------------- action */

/* eq. (18_6_4_1). Returns S; W[cls] = sum_n sum_{P in cls} Re tr P_n. */
double orc_action(const int32_t L[4], const double c[3], double beta, const cplx *U,
                  double W[3]) {
    lattice g = make_lattice(L);
    loop_t lp[34];
    int np = build_loops(lp);
    double *per = malloc(sizeof(double) * 3 * (size_t)g.V);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < g.V; ++n) {
        double w[3] = {0, 0, 0};
        for (int p = 0; p < np; ++p) w[lp[p].cls] += creal(m_trace(loop_product(&g, U, n, &lp[p])));
        for (int k = 0; k < 3; ++k) per[3 * n + k] = w[k];
    }
    ksum acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t n = 0; n < g.V; ++n)
        for (int k = 0; k < 3; ++k) ks_add(&acc[k], per[3 * n + k]);
    free(per);
    int count[3] = {0, 0, 0};
    for (int p = 0; p < np; ++p) count[lp[p].cls]++;
    ksum s = {0, 0};
    for (int k = 0; k < 3; ++k) {
        double wk = ks_val(&acc[k]);
        if (W) W[k] = wk;
        ks_add(&s, c[k] * 3.0 * (double)count[k] * (double)g.V);
        ks_add(&s, -c[k] * wk);
    }
    return beta / 3.0 * ks_val(&s);
}

/* ------------------------------------------------------------------- staples */

/*
 * The staple that loop p contributes through its l-th link to link (k,rho) when
 * d_l = +rho or -rho, following the algorithm after eq. (18_6_6_13):
 *   d_l = +rho: base n = k - sum_{j<l} d_j, staple = U_{n_{l+1}} ... U_{n_L} U_{n_1} ... U_{n_{l-1}};
 *   d_l = -rho: n_l = k + rho, base n = n_l - sum_{j<l} d_j,
 *               staple = U^dag_{n_{l-1}} ... U^dag_{n_1} U^dag_{n_L} ... U^dag_{n_{l+1}}.
 * Indices l are 0-based here. Also returns the base site through *base.
 */
static mat3 staple(const lattice *g, const cplx *U, int64_t k, int rho, const loop_t *p, int l,
                   int64_t *base) {
    int dl = p->d[l];
    int64_t n = (dl > 0) ? k : step(g, k, rho + 1); /* n_l */
    for (int j = l - 1; j >= 0; --j) n = step(g, n, -p->d[j]);
    if (base) *base = n;
    int64_t site[6];
    site[0] = n;
    for (int j = 1; j < p->len; ++j) site[j] = step(g, site[j - 1], p->d[j - 1]);
    mat3 r = m_unit();
    if (dl > 0) {
        for (int j = l + 1; j < p->len; ++j) r = m_mul(r, link(g, U, site[j], p->d[j]));
        for (int j = 0; j < l; ++j) r = m_mul(r, link(g, U, site[j], p->d[j]));
    } else {
        for (int j = l - 1; j >= 0; --j) r = m_mul(r, m_dag(link(g, U, site[j], p->d[j])));
        for (int j = p->len - 1; j > l; --j) r = m_mul(r, m_dag(link(g, U, site[j], p->d[j])));
    }
    return r;
}

/* t_{k,rho} split by loop class (unweighted), gathered link by link: every (loop,
 * position) pair whose link runs along +-rho names one staple of (k,rho). Used for
 * the force on a list of links; the whole field is built by the scatter below. */
static void staple_sums(const lattice *g, const cplx *U, const loop_t *lp, int np, int64_t k,
                        int rho, mat3 t[3]) {
    for (int c = 0; c < 3; ++c) t[c] = m_zero();
    for (int p = 0; p < np; ++p)
        for (int l = 0; l < lp[p].len; ++l)
            if (abs(lp[p].d[l]) == rho + 1)
                t[lp[p].cls] = m_add_scaled(t[lp[p].cls], 1.0, staple(g, U, k, rho, &lp[p], l, NULL));
}

static mat3 force_one(const lattice *g, const cplx *U, const loop_t *lp, int np,
                      const double c[3], double beta, int64_t k, int rho) {
    mat3 t[3];
    staple_sums(g, U, lp, np, k, rho, t);
    mat3 tw = m_zero();
    for (int cl = 0; cl < 3; ++cl) tw = m_add_scaled(tw, c[cl], t[cl]);
    mat3 u = m_load(U + (k * 4 + rho) * 9);
    return m_scale(m_ta(m_mul(u, tw)), beta / 6.0);
}

/*
 * Scatter form of the staple sums, written from the action itself (eq. 18_6_4_1) and
 * the derivative of eq. (18_7_25_2): every loop instance P_n = L_1 ... L_m is walked
 * once from its base site n, and for every position j the derivative of Re tr P_n
 * with respect to the link that L_j stands for is deposited into that link's t:
 *   tr P_n = tr(L_j A_j),  A_j = L_{j+1} ... L_m L_1 ... L_{j-1}  (cyclic order);
 *   d_j = +mu: L_j = U_{n_j,mu},            Re tr P_n = Re tr(U A_j),   deposit A_j   at (n_j, mu);
 *   d_j = -mu: L_j = U^dag_{n_j - mu, mu},  Re tr P_n = Re tr(U A_j^dag), deposit A_j^dag at (n_j - mu, mu).
 * acc holds ncls matrices per link, acc[((site*4 + mu)*ncls + slot)*9], where slot is
 * the loop's class (ncls = 3, weight 1) or 0 (ncls = 1, weight w[class]).
 */
static void deposit_loop(const lattice *g, const cplx *U, int64_t n, const loop_t *p, int ncls,
                         const double w[3], cplx *acc) {
    mat3 Lk[6];
    int64_t recv[6];
    int64_t s = n;
    for (int j = 0; j < p->len; ++j) {
        Lk[j] = link(g, U, s, p->d[j]);
        int64_t nx = step(g, s, p->d[j]);
        recv[j] = p->d[j] > 0 ? s * 4 + (p->d[j] - 1) : nx * 4 + (-p->d[j] - 1);
        s = nx;
    }
    const int slot = ncls == 1 ? 0 : p->cls;
    const double wt = ncls == 1 ? w[p->cls] : 1.0;
    for (int j = 0; j < p->len; ++j) {
        mat3 a = m_unit();
        for (int i = 1; i < p->len; ++i) a = m_mul(a, Lk[(j + i) % p->len]);
        if (p->d[j] < 0) a = m_dag(a);
        cplx *dst = acc + (recv[j] * ncls + slot) * 9;
        m_store(dst, m_add_scaled(m_load(dst), wt, a));
    }
}

/* Extent along t, relative to the base site, of the sites whose links a loop deposits to. */
static void deposit_t_extent(const loop_t *lp, int np, int *lo, int *hi) {
    *lo = 0;
    *hi = 0;
    for (int p = 0; p < np; ++p) {
        int t = 0;
        for (int j = 0; j < lp[p].len; ++j) {
            int d = lp[p].d[j];
            int nt = t + (d == 4 ? 1 : d == -4 ? -1 : 0);
            int r = d > 0 ? t : nt; /* receiving site of position j */
            if (r < *lo) *lo = r;
            if (r > *hi) *hi = r;
            t = nt;
        }
    }
}

/*
 * acc (zeroed by the caller) += the deposits of every loop instance. Base sites are
 * taken t-slice by t-slice in `nph` phases, nph the smallest divisor of Lt not below
 * the deposit extent: the slices of one phase are nph apart, deposit to disjoint
 * slices and run in parallel, and every link receives its deposits in the same order
 * whatever the thread count. Lattices too short in t for two slices per phase run
 * serially.
 */
static void scatter_staples(const lattice *g, const cplx *U, const loop_t *lp, int np, int ncls,
                            const double w[3], cplx *acc) {
    int lo, hi;
    deposit_t_extent(lp, np, &lo, &hi);
    const int Lt = g->L[3];
    int nph = hi - lo + 1;
    while (nph < Lt && Lt % nph != 0) ++nph;
    const int64_t per = g->V / Lt; /* sites per t-slice */
    if (Lt < 2 * nph) {
        for (int64_t n = 0; n < g->V; ++n)
            for (int p = 0; p < np; ++p) deposit_loop(g, U, n, &lp[p], ncls, w, acc);
        return;
    }
    for (int phase = 0; phase < nph; ++phase) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int q = 0; q < Lt / nph; ++q) {
            const int64_t t = (int64_t)q * nph + phase;
            for (int64_t n = t * per; n < (t + 1) * per; ++n)
                for (int p = 0; p < np; ++p) deposit_loop(g, U, n, &lp[p], ncls, w, acc);
        }
    }
}

/* G_{k,rho} = (beta/6)(U_{k,rho} t_{k,rho})_TA for every link, t from the scatter. */
void orc_force(const int32_t L[4], const double c[3], double beta, const cplx *U, cplx *G) {
    lattice g = make_lattice(L);
    loop_t lp[34];
    int np = build_loops(lp);
    memset(G, 0, sizeof(cplx) * 9 * 4 * (size_t)g.V);
    scatter_staples(&g, U, lp, np, 1, c, G);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < 4 * g.V; ++i)
        m_store(G + i * 9, m_scale(m_ta(m_mul(m_load(U + i * 9), m_load(G + i * 9))), beta / 6.0));
}

/* The same force for a list of links only, gathered link by link (sampled checks on
 * large lattices; a second formulation of the staple sums beside the scatter). */
void orc_force_links(const int32_t L[4], const double c[3], double beta, const cplx *U,
                     int64_t nlinks, const int64_t *site, const int32_t *mu, cplx *G) {
    lattice g = make_lattice(L);
    loop_t lp[34];
    int np = build_loops(lp);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nlinks; ++i)
        m_store(G + i * 9, force_one(&g, U, lp, np, c, beta, site[i], mu[i]));
}

/* Unweighted per-class staple sums t[cls] for every link: out[((k*4+rho)*3+cls)*9 ...]. */
void orc_staple_sums(const int32_t L[4], const cplx *U, cplx *out) {
    lattice g = make_lattice(L);
    loop_t lp[34];
    int np = build_loops(lp);
    const double one[3] = {1.0, 1.0, 1.0};
    memset(out, 0, sizeof(cplx) * 9 * 3 * 4 * (size_t)g.V);
    scatter_staples(&g, U, lp, np, 3, one, out);
}

/*
 * Part of S_G that depends on link (k,rho): beta/3 sum c_P [3 - Re tr P_n] over the
 * loop instances that contain the link (each (loop, position) pair with d_l = +-rho
 * names one instance through its base site). Used for finite differences on large
 * lattices, where differencing the extensive S would cancel most digits.
 */
double orc_local_action(const int32_t L[4], const double c[3], double beta, const cplx *U,
                        int64_t k, int32_t rho) {
    lattice g = make_lattice(L);
    loop_t lp[34];
    int np = build_loops(lp);
    ksum s = {0, 0};
    for (int p = 0; p < np; ++p)
        for (int l = 0; l < lp[p].len; ++l)
            if (abs(lp[p].d[l]) == rho + 1) {
                int64_t base;
                staple(&g, U, k, rho, &lp[p], l, &base);
                double rt = creal(m_trace(loop_product(&g, U, base, &lp[p])));
                ks_add(&s, c[lp[p].cls] * (3.0 - rt));
            }
    return beta / 3.0 * ks_val(&s);
}

/* --------------------------------------------------------- su(3) exponential */

/*
 * exp(X) by scaling and squaring of the Taylor series (Moler & Van Loan, "Nineteen
 * dubious ways", method 3): X/2^s with ||X/2^s||_1 <= 1/2, series summed until the
 * terms stop changing the result, then s squarings.
 */
static mat3 m_exp(mat3 x) {
    int s = 0;
    double nrm = m_norm1(x);
    while (nrm > 0.5) { nrm *= 0.5; ++s; }
    mat3 y = m_scale(x, ldexp(1.0, -s));
    mat3 sum = m_unit(), term = m_unit();
    for (int k = 1; k < 40; ++k) {
        term = m_scale(m_mul(term, y), 1.0 / k);
        sum = m_add_scaled(sum, 1.0, term);
        if (m_norm1(term) < 1e-18 * m_norm1(sum)) break;
    }
    for (int i = 0; i < s; ++i) sum = m_mul(sum, sum);
    return sum;
}

void orc_su3_exp(int64_t n, const cplx *X, cplx *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) m_store(out + 9 * i, m_exp(m_load(X + 9 * i)));
}

/* ---------------------------------------------------------- molecular dynamics */

/* sum over links of -tr(Pi^2) = sum (1/2) sum_a p_a^2 for Pi = i sum_a p_a T_a. */
double orc_kinetic(const int32_t L[4], const cplx *P) {
    lattice g = make_lattice(L);
    ksum s = {0, 0};
    for (int64_t i = 0; i < 4 * g.V; ++i) {
        mat3 p = m_load(P + 9 * i);
        ks_add(&s, -creal(m_trace(m_mul(p, p))));
    }
    return ks_val(&s);
}

/*
 * Leapfrog (position-momentum-position order of kicks: half kick, drift, half kick)
 * with Pi-dot = -G and U-dot = Pi U, where G = (beta/6)(U t)_TA and U = exp(i omega.T)
 * with dU/domega = iTU (Sec. II). The drift is U <- exp(dt Pi) U. H = kinetic + S_G.
 * U and P are updated in place; H_out[0] = H before, H_out[1] = H after.
 */
int orc_leapfrog(const int32_t L[4], const double c[3], double beta, cplx *U, cplx *P,
                 double dt, int32_t nsteps, double H_out[2]) {
    lattice g = make_lattice(L);
    int64_t nl = 4 * g.V;
    cplx *G = malloc(sizeof(cplx) * 9 * (size_t)nl);
    if (!G) return -1;
    H_out[0] = orc_kinetic(L, P) + orc_action(L, c, beta, U, NULL);
    for (int it = 0; it < nsteps; ++it) {
        orc_force(L, c, beta, U, G);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nl; ++i)
            m_store(P + 9 * i, m_add_scaled(m_load(P + 9 * i), -0.5 * dt, m_load(G + 9 * i)));
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nl; ++i) {
            mat3 e = m_exp(m_scale(m_load(P + 9 * i), dt));
            m_store(U + 9 * i, m_mul(e, m_load(U + 9 * i)));
        }
        orc_force(L, c, beta, U, G);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nl; ++i)
            m_store(P + 9 * i, m_add_scaled(m_load(P + 9 * i), -0.5 * dt, m_load(G + 9 * i)));
    }
    H_out[1] = orc_kinetic(L, P) + orc_action(L, c, beta, U, NULL);
    free(G);
    return 0;
}

/* Threads OpenMP would use (reported beside CPU timings). */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the calling thread's later parallel regions (timing at a chosen thread
 * count); n <= 0 leaves the setting unchanged. Returns the resulting count. */
int orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#endif
    return orc_num_threads();
}

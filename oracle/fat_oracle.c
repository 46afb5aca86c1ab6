/*
 * fat_oracle.c -- plain FP64 CPU oracle for the asqtad / HISQ fat-link smearing and
 * the force it induces on the thin links (the "path force").
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this library. It shares no code, header, table or helper with
 * the GPU library, and the GPU library never calls it.
 *
 * Source: D. Li, "The Calculation of Force in Lattice QCD", arXiv:1808.02281,
 * Sec. "Asqtad fermion" and Sec. "HISQ fermion":
 *
 *   - the paths of the asqtad matrix: one-link (eq. 18_6_6_3_1), three-staple
 *     (eq. 18_6_6_4), five-staple (eq. 18_6_6_5), seven-staple (eq. 18_6_6_6), Lepage
 *     (eq. 18_6_6_7) and Naik (eq. 18_6_6_3) terms, 688 oriented paths in all;
 *   - the fat link V_{p,mu} = sum over the smearing paths P from p to p+mu of
 *     c_P times the product of links along P (eq. 18_6_6_7_2), and the Naik long link
 *     W_{p,mu} = c_N U_{p,mu} U_{p+mu,mu} U_{p+2mu,mu};
 *   - the derivative of a function of V through the smearing: F~ of eq. 18_7_24_7.
 *     For the whole field every path instance is walked once and deposits, at each of
 *     its links, the derivative of its trace with respect to that link (scatter);
 *     single links are gathered by the enumerated algorithm after eq. 18_7_24_7 (for
 *     every path link along +-rho: A = product of the links before it, B = product of
 *     the links after it times F^T). The two formulations are checked against each
 *     other.
 *
 * What is differentiated: the real scalar
 *     Phi(U) = Re sum_{p,mu} tr(GV_{p,mu}^dagger V_{p,mu}) + Re sum tr(GW^dagger W)
 * for given per-link matrices GV, GW. GV is the paper's F of eq. 18_7_24_4 complex-
 * conjugated (F^T = GV^dagger), so that Phi is the real part of the paper's
 * contraction F_{ef} V_{ef}; the staggered phases eta and the outer products of the
 * fermion fields are carried by GV. The result is the gradient
 *     grad_{k,rho} = dPhi/dRe U_{k,rho} + i dPhi/dIm U_{k,rho},
 * i.e. dPhi = Re sum tr(grad^dagger dU) for any complex variation dU; it equals the
 * complex conjugate of the paper's F~. For a path link that is traversed forwards
 * (d_l = +rho) the paper's product R = B A = U_{l+1}..U_L F^T U_1..U_{l-1} enters as
 * R^dagger; for a link traversed backwards (d_l = -rho, the matrix U^dagger_{k,rho})
 * it enters as R itself: the paper's derivative rule for d_l = -rho is read as acting
 * on the conjugate link (a reading pinned by finite differences in the tests).
 *
 * The force on the thin links in the convention of the gauge force of Sec. II
 * (dPhi/domega^a_{k,rho} = -2i tr(T_a G) for U -> exp(i omega.T) U) is
 *     G_{k,rho} = -(1/2) (U_{k,rho} grad_{k,rho}^dagger)_TA      (eq. 18_7_24_6).
 *
 * Coefficients c[6] = {c_1, c_3, c_5, c_7, c_L, c_N} are inputs; the paper gives no
 * values. Layout: canonical AoS lexicographic, as in sym_oracle.c.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;
typedef struct { cplx a[3][3]; } mat3;

static mat3 z3(void) { mat3 r; memset(&r, 0, sizeof r); return r; }

static mat3 one3(void) {
    mat3 r = z3();
    for (int i = 0; i < 3; ++i) r.a[i][i] = 1.0;
    return r;
}

static mat3 mul3(mat3 x, mat3 y) {
    mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += x.a[i][k] * y.a[k][j];
            r.a[i][j] = s;
        }
    return r;
}

static mat3 dag3(mat3 x) {
    mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = conj(x.a[j][i]);
    return r;
}

static mat3 axpy3(mat3 y, double c, mat3 x) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) y.a[i][j] += c * x.a[i][j];
    return y;
}

static mat3 ld3(const cplx *p) {
    mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = p[3 * i + j];
    return r;
}

static void st3(cplx *p, mat3 x) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) p[3 * i + j] = x.a[i][j];
}

/* antihermitian traceless part: (B - B^dagger)/2 - tr(B - B^dagger)/6 (eq. 18_6_6_11) */
static mat3 ta3(mat3 b) {
    mat3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = 0.5 * (b.a[i][j] - conj(b.a[j][i]));
    cplx tr = (r.a[0][0] + r.a[1][1] + r.a[2][2]) / 3.0;
    for (int i = 0; i < 3; ++i) r.a[i][i] -= tr;
    return r;
}

/* ------------------------------------------------------------------ geometry */

typedef struct { int L[4]; int64_t V; } lat;

static lat mklat(const int32_t L[4]) {
    lat g;
    g.V = 1;
    for (int m = 0; m < 4; ++m) { g.L[m] = L[m]; g.V *= L[m]; }
    return g;
}

/* n + d-hat for a signed direction d in {+-1..+-4} (axis |d|-1), periodic. */
static int64_t hop(const lat *g, int64_t s, int d) {
    int x[4];
    int64_t r = s;
    for (int m = 0; m < 4; ++m) { x[m] = (int)(r % g->L[m]); r /= g->L[m]; }
    int m = abs(d) - 1;
    x[m] = (x[m] + (d > 0 ? 1 : g->L[m] - 1)) % g->L[m];
    int64_t out = 0;
    for (int k = 3; k >= 0; --k) out = out * g->L[k] + x[k];
    return out;
}

/* U_{n,d}, with U_{n,-mu} = U^dagger_{n-mu,mu} */
static mat3 lnk(const lat *g, const cplx *U, int64_t n, int d) {
    if (d > 0) return ld3(U + (n * 4 + (d - 1)) * 9);
    return dag3(ld3(U + (hop(g, n, d) * 4 + (-d - 1)) * 9));
}

/* ------------------------------------------------------------------- paths */

enum { FAT_ONE = 0, FAT_3 = 1, FAT_5 = 2, FAT_7 = 3, FAT_LEPAGE = 4, FAT_NAIK = 5 };
#define FAT_NPATH 85
#define FAT_MAXLEN 7

typedef struct { int len; int cls; int d[FAT_MAXLEN]; } fpath;

/* The smearing paths from p to p + mu-hat (mu = 1..4) of eq. 18_6_6_7_2, with the
 * Lepage term of eq. 18_6_6_7: one-link, three-staples (nu != mu, both signs),
 * five-staples (ordered nu != rho, both != mu, all four sign pairs), seven-staples
 * (ordered distinct nu, rho, sigma != mu, all eight sign triples), Lepage
 * (nu != mu, both signs, two steps out and two back). */
static int fat_paths(int mu, fpath out[FAT_NPATH]) {
    int n = 0;
    fpath p;
    memset(&p, 0, sizeof p);
    p.len = 1; p.cls = FAT_ONE; p.d[0] = mu;
    out[n++] = p;
    for (int nu = 1; nu <= 4; ++nu) {
        if (nu == mu) continue;
        for (int s = -1; s <= 1; s += 2) {
            fpath q = {3, FAT_3, {s * nu, mu, -s * nu}};
            out[n++] = q;
        }
    }
    for (int nu = 1; nu <= 4; ++nu)
        for (int rho = 1; rho <= 4; ++rho) {
            if (nu == mu || rho == mu || rho == nu) continue;
            for (int s1 = -1; s1 <= 1; s1 += 2)
                for (int s2 = -1; s2 <= 1; s2 += 2) {
                    fpath q = {5, FAT_5, {s1 * nu, s2 * rho, mu, -s2 * rho, -s1 * nu}};
                    out[n++] = q;
                }
        }
    for (int nu = 1; nu <= 4; ++nu)
        for (int rho = 1; rho <= 4; ++rho)
            for (int sg = 1; sg <= 4; ++sg) {
                if (nu == mu || rho == mu || sg == mu || rho == nu || sg == nu || sg == rho) continue;
                for (int s1 = -1; s1 <= 1; s1 += 2)
                    for (int s2 = -1; s2 <= 1; s2 += 2)
                        for (int s3 = -1; s3 <= 1; s3 += 2) {
                            fpath q = {7, FAT_7,
                                       {s1 * nu, s2 * rho, s3 * sg, mu, -s3 * sg, -s2 * rho, -s1 * nu}};
                            out[n++] = q;
                        }
            }
    for (int nu = 1; nu <= 4; ++nu) {
        if (nu == mu) continue;
        for (int s = -1; s <= 1; s += 2) {
            fpath q = {5, FAT_LEPAGE, {s * nu, s * nu, mu, -s * nu, -s * nu}};
            out[n++] = q;
        }
    }
    return n;
}

/* Path table for direction mu = 0..3 (the Naik path last): returns the count (86). */
int orc_fat_paths(int32_t mu, int32_t *len, int32_t *cls, int32_t *dirs /* 86 x 7 */) {
    fpath P[FAT_NPATH];
    int n = fat_paths(mu + 1, P);
    for (int i = 0; i < n; ++i) {
        len[i] = P[i].len;
        cls[i] = P[i].cls;
        for (int j = 0; j < FAT_MAXLEN; ++j) dirs[i * FAT_MAXLEN + j] = j < P[i].len ? P[i].d[j] : 0;
    }
    len[n] = 3;
    cls[n] = FAT_NAIK;
    for (int j = 0; j < FAT_MAXLEN; ++j) dirs[n * FAT_MAXLEN + j] = j < 3 ? mu + 1 : 0;
    return n + 1;
}

static mat3 walk(const lat *g, const cplx *U, int64_t p, const int *d, int from, int to, int64_t *site) {
    /* product of the links from position `from` to `to` - 1 of the path starting at p */
    mat3 r = one3();
    int64_t s = p;
    for (int j = 0; j < from; ++j) s = hop(g, s, d[j]);
    for (int j = from; j < to; ++j) {
        r = mul3(r, lnk(g, U, s, d[j]));
        s = hop(g, s, d[j]);
    }
    if (site) *site = s;
    return r;
}

/* V and W of every link. W may be NULL. */
void orc_fat_links(const int32_t L[4], const double c[6], const cplx *U, cplx *V, cplx *W) {
    lat g = mklat(L);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < g.V; ++p) {
        for (int mu = 1; mu <= 4; ++mu) {
            fpath P[FAT_NPATH];
            int np = fat_paths(mu, P);
            mat3 v = z3();
            for (int i = 0; i < np; ++i) v = axpy3(v, c[P[i].cls], walk(&g, U, p, P[i].d, 0, P[i].len, NULL));
            st3(V + (p * 4 + (mu - 1)) * 9, v);
            if (W) {
                const int nk[3] = {mu, mu, mu};
                mat3 w = walk(&g, U, p, nk, 0, 3, NULL);
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) w.a[i][j] *= c[FAT_NAIK];
                st3(W + (p * 4 + (mu - 1)) * 9, w);
            }
        }
    }
}

/* Contribution of every path through the link (k, rho) -- the algorithm after
 * eq. 18_7_24_7 with its loops ordered by the link that receives the contribution. */
static mat3 grad_one(const lat *g, const double c[6], const cplx *U, const cplx *GV, const cplx *GW,
                     int64_t k, int rho /* 1..4 */) {
    mat3 acc = z3();
    for (int mu = 1; mu <= 4; ++mu) {
        fpath P[FAT_NPATH + 1];
        int np = fat_paths(mu, P);
        fpath naik = {3, FAT_NAIK, {mu, mu, mu}};
        P[np++] = naik;
        for (int i = 0; i < np; ++i) {
            const fpath *q = &P[i];
            const cplx *G = q->cls == FAT_NAIK ? GW : GV;
            if (G == NULL) continue;
            for (int l = 0; l < q->len; ++l) {
                if (abs(q->d[l]) != rho) continue;
                /* n_l: the site the l-th step starts from */
                int64_t nl = q->d[l] > 0 ? k : hop(g, k, rho);
                int64_t p = nl;
                for (int j = l - 1; j >= 0; --j) p = hop(g, p, -q->d[j]);
                mat3 A = walk(g, U, p, q->d, 0, l, NULL);             /* U_1 ... U_{l-1} */
                mat3 B = walk(g, U, p, q->d, l + 1, q->len, NULL);    /* U_{l+1} ... U_L */
                mat3 Ft = dag3(ld3(G + (p * 4 + (mu - 1)) * 9));      /* F^T = G^dagger */
                mat3 R = mul3(mul3(B, Ft), A);
                R = q->d[l] > 0 ? dag3(R) : R;
                acc = axpy3(acc, c[q->cls], R);
            }
        }
    }
    return acc;
}

/*
 * Scatter form of the same gradient for the whole field, written from the definition
 * of Phi: every path instance (base p, direction mu, path q) is walked once, links
 * L_1 ... L_m, and for every position l
 *     c_q tr(F^T L_1 ... L_m) = c_q tr(L_l R),  R = (L_{l+1} ... L_m) F^T (L_1 ... L_{l-1}),
 * so dPhi = Re tr(grad^dagger dU) receives R^dagger at the link (n_l, rho) when
 * d_l = +rho (L_l = U) and R at (n_l - rho, rho) when d_l = -rho (L_l = U^dagger).
 */
static void fat_deposit(const lat *g, const double c[6], const cplx *U, const cplx *G, int64_t p, int mu,
                        const fpath *q, cplx *acc) {
    mat3 Lk[FAT_MAXLEN];
    int64_t recv[FAT_MAXLEN];
    int64_t s = p;
    for (int j = 0; j < q->len; ++j) {
        Lk[j] = lnk(g, U, s, q->d[j]);
        int64_t nx = hop(g, s, q->d[j]);
        recv[j] = q->d[j] > 0 ? s * 4 + (q->d[j] - 1) : nx * 4 + (-q->d[j] - 1);
        s = nx;
    }
    const mat3 Ft = dag3(ld3(G + (p * 4 + (mu - 1)) * 9));
    for (int l = 0; l < q->len; ++l) {
        mat3 R = one3();
        for (int j = l + 1; j < q->len; ++j) R = mul3(R, Lk[j]);
        R = mul3(R, Ft);
        for (int j = 0; j < l; ++j) R = mul3(R, Lk[j]);
        if (q->d[l] > 0) R = dag3(R);
        st3(acc + recv[l] * 9, axpy3(ld3(acc + recv[l] * 9), c[q->cls], R));
    }
}

/* Extent along t, relative to the base site, of the sites whose links the paths of
 * every direction (the Naik path included) deposit to. */
static void fat_t_extent(int *lo, int *hi) {
    *lo = 0;
    *hi = 0;
    for (int mu = 1; mu <= 4; ++mu) {
        fpath P[FAT_NPATH + 1];
        int np = fat_paths(mu, P);
        fpath naik = {3, FAT_NAIK, {mu, mu, mu}};
        P[np++] = naik;
        for (int i = 0; i < np; ++i) {
            int t = 0;
            for (int j = 0; j < P[i].len; ++j) {
                int d = P[i].d[j];
                int nt = t + (d == 4 ? 1 : d == -4 ? -1 : 0);
                int r = d > 0 ? t : nt;
                if (r < *lo) *lo = r;
                if (r > *hi) *hi = r;
                t = nt;
            }
        }
    }
}

static void fat_deposit_site(const lat *g, const double c[6], const cplx *U, const cplx *GV, const cplx *GW,
                             int64_t p, cplx *acc) {
    for (int mu = 1; mu <= 4; ++mu) {
        fpath P[FAT_NPATH];
        int np = fat_paths(mu, P);
        for (int i = 0; i < np; ++i) fat_deposit(g, c, U, GV, p, mu, &P[i], acc);
        if (GW != NULL) {
            fpath naik = {3, FAT_NAIK, {mu, mu, mu}};
            fat_deposit(g, c, U, GW, p, mu, &naik, acc);
        }
    }
}

/* grad_{k,rho} for every link (GW may be NULL: no Naik term), by the scatter above.
 * Base sites go t-slice by t-slice in phases whose slices are far enough apart to
 * deposit to disjoint slices (parallel inside a phase, the same order of deposits at
 * every link whatever the thread count); lattices short in t run serially. */
void orc_fat_grad(const int32_t L[4], const double c[6], const cplx *U, const cplx *GV, const cplx *GW,
                  cplx *grad) {
    lat g = mklat(L);
    memset(grad, 0, sizeof(cplx) * 9 * 4 * (size_t)g.V);
    int lo, hi;
    fat_t_extent(&lo, &hi);
    const int Lt = g.L[3];
    int nph = hi - lo + 1;
    while (nph < Lt && Lt % nph != 0) ++nph;
    const int64_t per = g.V / Lt;
    if (Lt < 2 * nph) {
        for (int64_t p = 0; p < g.V; ++p) fat_deposit_site(&g, c, U, GV, GW, p, grad);
        return;
    }
    for (int phase = 0; phase < nph; ++phase) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int q = 0; q < Lt / nph; ++q) {
            const int64_t t = (int64_t)q * nph + phase;
            for (int64_t p = t * per; p < (t + 1) * per; ++p) fat_deposit_site(&g, c, U, GV, GW, p, grad);
        }
    }
}

/* grad for a list of links (site, mu) only; out is (n, 3, 3). */
void orc_fat_grad_links(const int32_t L[4], const double c[6], const cplx *U, const cplx *GV, const cplx *GW,
                        int64_t n, const int64_t *sites, const int32_t *mus, cplx *out) {
    lat g = mklat(L);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) st3(out + i * 9, grad_one(&g, c, U, GV, GW, sites[i], mus[i] + 1));
}

/* G = -(1/2)(U grad^dagger)_TA per link: the force in the gauge-force convention. */
void orc_fat_force_from_grad(int64_t nlinks, const cplx *U, const cplx *grad, cplx *G) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nlinks; ++k) {
        mat3 t = ta3(mul3(ld3(U + k * 9), dag3(ld3(grad + k * 9))));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) t.a[i][j] *= -0.5;
        st3(G + k * 9, t);
    }
}

/* V and W of a list of links (site, mu) only; out shapes (n, 3, 3). W may be NULL. */
void orc_fat_links_links(const int32_t L[4], const double c[6], const cplx *U, int64_t n, const int64_t *sites,
                         const int32_t *mus, cplx *V, cplx *W) {
    lat g = mklat(L);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        int mu = mus[i] + 1;
        fpath P[FAT_NPATH];
        int np = fat_paths(mu, P);
        mat3 v = z3();
        for (int k = 0; k < np; ++k) v = axpy3(v, c[P[k].cls], walk(&g, U, sites[i], P[k].d, 0, P[k].len, NULL));
        st3(V + i * 9, v);
        if (W) {
            const int nk[3] = {mu, mu, mu};
            mat3 w = walk(&g, U, sites[i], nk, 0, 3, NULL);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) w.a[a][b] *= c[FAT_NAIK];
            st3(W + i * 9, w);
        }
    }
}

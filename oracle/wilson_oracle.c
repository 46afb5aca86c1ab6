/*
 * wilson_oracle.c -- plain FP64 CPU oracle for the Wilson fermion matrix with clover
 * term and the fermion force it gives for fixed vectors X, Y.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this library. It shares no code, header, table or helper with
 * the GPU library, and the GPU library never calls it.
 *
 * Source: D. Li, "The Calculation of Force in Lattice QCD", arXiv:1808.02281,
 * Sec. "Wilson fermion action with clover term":
 *   - D = A - kappa Dh (eq. 18_7_17_2), hopping part Dh of eq. 18_7_17_4 with the
 *     projectors (1 - gamma_mu) forwards and (1 + gamma_mu) backwards;
 *   - clover diagonal A_n = 1 - c_sw/(32(m+4)) sum_{mu != nu} [gamma_mu, gamma_nu] Q_{n;mu nu}
 *     (eq. 18_7_18_0), kappa = 1/(2(m+4)) so that c_sw/(32(m+4)) = c_sw kappa / 16, with
 *     the clover leaves Q of eq. 17_7_20_8;
 *   - for fixed X, Y (in the paper X = (D^+ D)^{-1} phi, Y = D X, eq. 18_6_24_0_1) the
 *     derivative Y^+ dD/domega X + c.c. (eq. 18_6_24_0): hopping part from the outer
 *     products B and C of eqs. 18_1_29_20_2 and 18_1_29_20_3; clover part from
 *     eq. 18_7_17_31 with the sites n = k, k+rho, k+-nu, k+rho+-nu and the rule of
 *     eqs. 18_7_26_9, 18_7_26_10 (the derivative puts i T before U_{k,rho} and splits
 *     each leaf term into two vectors contracted over spin).
 *
 * What is computed: Psi(U) = Y^+ D X + c.c. = 2 Re Y^+ D X. Its derivative along
 * U_{k,rho} -> exp(i omega.T) U_{k,rho} is written Re tr(i T_a M_{k,rho}) and returned as
 *     G_{k,rho} = -(1/2) (M_{k,rho})_TA,   so that   dPsi/domega^a = -2i tr(T_a G),
 * the convention of the gauge force G of Sec. II. By eq. 18_6_24_0 the pseudofermion
 * action at fixed X, Y changes by -dPsi, so its force in that convention is -G.
 *
 * Readings: gamma matrices are Hermitian
 * in the DeGrand-Rossi basis, gamma_1..gamma_4 for the x, y, z, t directions; the
 * paper's leaf products U_{n;mu,nu} are plaquettes starting at n (first step mu,
 * second nu); spinors are AoS (Lt,Lz,Ly,Lx,4,3): site, spin, colour.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;
typedef struct { cplx a[3][3]; } m3;
typedef struct { cplx v[4][3]; } spinor; /* [spin][colour] */

static m3 mz(void) { m3 r; memset(&r, 0, sizeof r); return r; }
static m3 mone(void) { m3 r = mz(); for (int i = 0; i < 3; ++i) r.a[i][i] = 1; return r; }
static m3 mmul(m3 x, m3 y) {
    m3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += x.a[i][k] * y.a[k][j];
            r.a[i][j] = s;
        }
    return r;
}
static m3 mdag(m3 x) {
    m3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = conj(x.a[j][i]);
    return r;
}
static m3 mld(const cplx *p) {
    m3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = p[3 * i + j];
    return r;
}
static void mst(cplx *p, m3 x) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) p[3 * i + j] = x.a[i][j];
}
static spinor sld(const cplx *p) {
    spinor s;
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) s.v[a][c] = p[3 * a + c];
    return s;
}

/* ------------------------------------------------------------ Dirac algebra */

/* Hermitian gamma matrices, DeGrand-Rossi basis; mu = 0..3 for x, y, z, t. */
static void gamma_mat(int mu, cplx g[4][4]) {
    memset(g, 0, sizeof(cplx) * 16);
    switch (mu) {
        case 0: g[0][3] = I; g[1][2] = I; g[2][1] = -I; g[3][0] = -I; break;
        case 1: g[0][3] = -1; g[1][2] = 1; g[2][1] = 1; g[3][0] = -1; break;
        case 2: g[0][2] = I; g[1][3] = -I; g[2][0] = -I; g[3][1] = I; break;
        default: g[0][2] = 1; g[1][3] = 1; g[2][0] = 1; g[3][1] = 1; break;
    }
}

void orc_gamma(int32_t mu, cplx *out /* 4x4 */) {
    cplx g[4][4];
    gamma_mat(mu, g);
    memcpy(out, g, sizeof g);
}

/* [gamma_mu, gamma_nu] */
static void commutator(int mu, int nu, cplx c[4][4]) {
    cplx a[4][4], b[4][4];
    gamma_mat(mu, a);
    gamma_mat(nu, b);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += a[i][k] * b[k][j] - b[i][k] * a[k][j];
            c[i][j] = s;
        }
}

/* (1 + sgn gamma_mu) applied in spin space */
static spinor proj(int mu, int sgn, spinor x) {
    cplx g[4][4];
    gamma_mat(mu, g);
    spinor r;
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) {
            cplx s = x.v[a][c];
            for (int b = 0; b < 4; ++b) s += sgn * g[a][b] * x.v[b][c];
            r.v[a][c] = s;
        }
    return r;
}

static spinor spin_mat(cplx g[4][4], spinor x) {
    spinor r;
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) {
            cplx s = 0;
            for (int b = 0; b < 4; ++b) s += g[a][b] * x.v[b][c];
            r.v[a][c] = s;
        }
    return r;
}

static spinor colour(m3 u, spinor x) {
    spinor r;
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += u.a[i][k] * x.v[a][k];
            r.v[a][i] = s;
        }
    return r;
}

/* sum over spin of the colour outer product: out_{ba} = sum_alpha p_{alpha b} conj(q_{alpha a}) */
static m3 outer(spinor p, spinor q) {
    m3 r;
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
            cplx s = 0;
            for (int al = 0; al < 4; ++al) s += p.v[al][b] * conj(q.v[al][a]);
            r.a[b][a] = s;
        }
    return r;
}

/* ------------------------------------------------------------------ geometry */

typedef struct { int L[4]; int64_t V; } wlat;

static wlat wmk(const int32_t L[4]) {
    wlat g;
    g.V = 1;
    for (int m = 0; m < 4; ++m) { g.L[m] = L[m]; g.V *= L[m]; }
    return g;
}

static int64_t whop(const wlat *g, int64_t s, int d) {
    int x[4];
    int64_t r = s;
    for (int m = 0; m < 4; ++m) { x[m] = (int)(r % g->L[m]); r /= g->L[m]; }
    int m = abs(d) - 1;
    x[m] = (x[m] + (d > 0 ? 1 : g->L[m] - 1)) % g->L[m];
    int64_t out = 0;
    for (int k = 3; k >= 0; --k) out = out * g->L[k] + x[k];
    return out;
}

static m3 wlink(const wlat *g, const cplx *U, int64_t n, int d) {
    if (d > 0) return mld(U + (n * 4 + (d - 1)) * 9);
    return mdag(mld(U + (whop(g, n, d) * 4 + (-d - 1)) * 9));
}

/* The leaf U_{n;d1,d2} = U_{n,d1} U_{n+d1,d2} U_{n+d1+d2,-d1} U_{n+d2,-d2} (signed d). */
static void leaf_dirs(int d1, int d2, int d[4]) { d[0] = d1; d[1] = d2; d[2] = -d1; d[3] = -d2; }

/* The four leaves of Q_{n;mu nu} (eq. 17_7_20_8), mu, nu = 1..4 */
static void q_leaves(int mu, int nu, int d[4][4]) {
    leaf_dirs(mu, nu, d[0]);
    leaf_dirs(nu, -mu, d[1]);
    leaf_dirs(-mu, -nu, d[2]);
    leaf_dirs(-nu, mu, d[3]);
}

static m3 path(const wlat *g, const cplx *U, int64_t n, const int *d, int from, int to) {
    m3 r = mone();
    int64_t s = n;
    for (int j = 0; j < from; ++j) s = whop(g, s, d[j]);
    for (int j = from; j < to; ++j) {
        r = mmul(r, wlink(g, U, s, d[j]));
        s = whop(g, s, d[j]);
    }
    return r;
}

static m3 q_leaf_sum(const wlat *g, const cplx *U, int64_t n, int mu, int nu) {
    int d[4][4];
    q_leaves(mu, nu, d);
    m3 q = mz();
    for (int l = 0; l < 4; ++l) {
        m3 p = path(g, U, n, d[l], 0, 4);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) q.a[i][j] += p.a[i][j];
    }
    return q;
}

/* Q_{n;mu nu} for every site and ordered pair (mu, nu = 0..3; zero for mu == nu): (V,4,4,3,3) */
void orc_clover_leaves(const int32_t L[4], const cplx *U, cplx *Q) {
    wlat g = wmk(L);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < g.V; ++n)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = 0; nu < 4; ++nu)
                mst(Q + ((n * 4 + mu) * 4 + nu) * 9, mu == nu ? mz() : q_leaf_sum(&g, U, n, mu + 1, nu + 1));
}

/* ------------------------------------------------------------- matrix, Psi */

/* out = D X on every site (eq. 18_7_17_2 with A of eq. 18_7_18_0) */
void orc_wilson_apply(const int32_t L[4], double kappa, double csw, const cplx *U, const cplx *X, cplx *out) {
    wlat g = wmk(L);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < g.V; ++n) {
        spinor x = sld(X + n * 12);
        spinor r = x;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = 0; nu < 4; ++nu) {
                if (mu == nu) continue;
                cplx c[4][4];
                commutator(mu, nu, c);
                spinor t = colour(q_leaf_sum(&g, U, n, mu + 1, nu + 1), spin_mat(c, x));
                for (int a = 0; a < 4; ++a)
                    for (int k = 0; k < 3; ++k) r.v[a][k] -= csw * kappa / 16.0 * t.v[a][k];
            }
        for (int mu = 0; mu < 4; ++mu) {
            spinor f = proj(mu, -1, colour(wlink(&g, U, n, mu + 1), sld(X + whop(&g, n, mu + 1) * 12)));
            spinor b = proj(mu, +1, colour(wlink(&g, U, n, -(mu + 1)), sld(X + whop(&g, n, -(mu + 1)) * 12)));
            for (int a = 0; a < 4; ++a)
                for (int k = 0; k < 3; ++k) r.v[a][k] -= kappa * (f.v[a][k] + b.v[a][k]);
        }
        for (int a = 0; a < 4; ++a)
            for (int k = 0; k < 3; ++k) out[n * 12 + 3 * a + k] = r.v[a][k];
    }
}

/* Psi = 2 Re sum_n Y_n^+ (D X)_n */
double orc_wilson_psi(const int32_t L[4], double kappa, double csw, const cplx *U, const cplx *X, const cplx *Y) {
    wlat g = wmk(L);
    cplx *DX = (cplx *)malloc(sizeof(cplx) * 12 * (size_t)g.V);
    if (!DX) return NAN;
    orc_wilson_apply(L, kappa, csw, U, X, DX);
    double s = 0.0;
    for (int64_t i = 0; i < 12 * g.V; ++i) s += creal(conj(Y[i]) * DX[i]);
    free(DX);
    return 2.0 * s;
}

/* ------------------------------------------------------------------ force */

/* M_{k,rho} with dPsi/domega^a = Re tr(i T_a M) */
static m3 force_matrix(const wlat *g, double kappa, double csw, const cplx *U, const cplx *X, const cplx *Y,
                       int64_t k, int rho /* 0..3 */) {
    m3 M = mz();
    const m3 u = mld(U + (k * 4 + rho) * 9);
    const int64_t kr = whop(g, k, rho + 1);

    /* hopping (eqs. 18_1_29_20_1..3): Y^+ dD X = -kappa tr(i T (B - C)) */
    {
        spinor Z = proj(rho, -1, colour(u, sld(X + kr * 12)));                 /* (1 - g) U X_{k+rho} */
        m3 B = outer(Z, sld(Y + k * 12));
        spinor Wv = colour(u, proj(rho, +1, sld(Y + kr * 12)));                 /* U (1 + g) Y_{k+rho} */
        m3 C = outer(sld(X + k * 12), Wv);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M.a[i][j] += 2.0 * (-kappa) * (B.a[i][j] - C.a[i][j]);
    }

    /* clover (eq. 18_7_17_31): -c_sw kappa/16 sum_nu Y_n^+ [g_rho, g_nu] d(Q_{n;rho nu} - Q_{n;nu rho}) X_n
     * over n in {k, k+rho, k+-nu, k+rho+-nu}. Each leaf through the link is split at the link
     * (eqs. 18_7_26_9, 18_7_26_10): for a leaf P = A U_{k,rho} B from n, the term
     * Y^+ G A (iT U) B X is tr(iT (U B X) (x) (Y^+ G A)); for P = A U_{k,rho}^+ B it is
     * -tr(iT (B X) (x) (Y^+ G A U^+)). */
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == rho) continue;
        cplx cm[4][4];
        commutator(rho, nu, cm);
        int64_t sites[6];
        sites[0] = k;
        sites[1] = kr;
        sites[2] = whop(g, k, nu + 1);
        sites[3] = whop(g, k, -(nu + 1));
        sites[4] = whop(g, kr, nu + 1);
        sites[5] = whop(g, kr, -(nu + 1));
        for (int si = 0; si < 6; ++si) {
            const int64_t n = sites[si];
            /* on tiny lattices two entries of the list can be the same site */
            int dup = 0;
            for (int sj = 0; sj < si; ++sj) dup |= sites[sj] == n;
            if (dup) continue;
            spinor x = sld(X + n * 12);
            spinor y = sld(Y + n * 12);
            for (int ord = 0; ord < 2; ++ord) {
                const int a1 = ord == 0 ? rho + 1 : nu + 1, a2 = ord == 0 ? nu + 1 : rho + 1;
                const double sgn = ord == 0 ? 1.0 : -1.0; /* Q_{rho nu} - Q_{nu rho} */
                int d[4][4];
                q_leaves(a1, a2, d);
                for (int lf = 0; lf < 4; ++lf) {
                    int64_t s = n;
                    for (int l = 0; l < 4; ++l) {
                        const int dl = d[lf][l];
                        const int64_t nxt = whop(g, s, dl);
                        const int fwd = dl == rho + 1 && s == k;
                        const int bwd = dl == -(rho + 1) && nxt == k;
                        if (fwd || bwd) {
                            m3 A = path(g, U, n, d[lf], 0, l);
                            m3 Bp = path(g, U, n, d[lf], l + 1, 4);
                            /* Y^+ G A: as a spinor q with q^+ = Y^+ G A, i.e. q = A^+ G^+ Y */
                            cplx gd[4][4];
                            for (int i = 0; i < 4; ++i)
                                for (int j = 0; j < 4; ++j) gd[i][j] = conj(cm[j][i]);
                            spinor q = colour(mdag(A), spin_mat(gd, y));
                            m3 T;
                            if (fwd) {
                                spinor p = colour(u, colour(Bp, x)); /* U B X */
                                T = outer(p, q);
                            } else {
                                spinor p = colour(Bp, x);            /* B X */
                                spinor qq = colour(u, q);            /* (Y^+ G A U^+)^+ = U q */
                                T = outer(p, qq);
                                for (int i = 0; i < 3; ++i)
                                    for (int j = 0; j < 3; ++j) T.a[i][j] = -T.a[i][j];
                            }
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j) M.a[i][j] += 2.0 * (-csw * kappa / 16.0) * sgn * T.a[i][j];
                        }
                        s = nxt;
                    }
                }
            }
        }
    }
    return M;
}

static void store_force(cplx *out, m3 M) {
    m3 r;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] = 0.5 * (M.a[i][j] - conj(M.a[j][i]));
    cplx tr = (r.a[0][0] + r.a[1][1] + r.a[2][2]) / 3.0;
    for (int i = 0; i < 3; ++i) r.a[i][i] -= tr;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r.a[i][j] *= -0.5;
    mst(out, r);
}

/* G = -(1/2) M_TA on every link, AoS (V,4,3,3) */
void orc_wilson_force(const int32_t L[4], double kappa, double csw, const cplx *U, const cplx *X, const cplx *Y,
                      cplx *G) {
    wlat g = wmk(L);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t l = 0; l < g.V * 4; ++l)
        store_force(G + l * 9, force_matrix(&g, kappa, csw, U, X, Y, l / 4, (int)(l % 4)));
}

void orc_wilson_force_links(const int32_t L[4], double kappa, double csw, const cplx *U, const cplx *X,
                            const cplx *Y, int64_t n, const int64_t *sites, const int32_t *mus, cplx *G) {
    wlat g = wmk(L);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) store_force(G + i * 9, force_matrix(&g, kappa, csw, U, X, Y, sites[i], mus[i]));
}

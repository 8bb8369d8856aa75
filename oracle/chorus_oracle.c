/*
 * CPU FP64 oracle of the SD residual + SSP-RK3 update (test infrastructure;
 * see chorus_oracle.h).  Plain loops in the order of the method's steps:
 *
 *   Section 3  (1D operators)      solution points (Chebyshev-Gauss), flux
 *                                  points (Legendre-Gauss roots of P_{N-1}
 *                                  from the three-term recursion, plus 0, 1),
 *                                  Lagrange bases h_s and l_{m}.
 *   Section 3  (mapping)           20-node isoparametric map, |J|, and the
 *                                  transformed fluxes |J| J^{-1} (F, G, H).
 *   Section 3  (reconstruction)    tensor-product interpolation of Q to the
 *                                  flux points, Rusanov common inviscid flux,
 *                                  BR1-type averaging for the viscous terms,
 *                                  derivative of the flux polynomial.
 *   Section 2  (Eqs. 4-9)          fluxes F_inv, F_v, source M.
 *   Section 5                      impermeable, stress-free walls with exact
 *                                  inviscid wall flux.
 *   Section 4.2                    polytropic adiabatic reference state.
 *
 * Readings where the paper is silent or garbled (each is listed with its
 * reason in the design notes of the repository):
 *   - M uses g_vec = +GM x / r^3 (outward components of the magnitude), so
 *     that -M reproduces rho g and rho u.g of Eqs. 2-3; Coriolis as printed.
 *   - energy component of F_v is u.tau - f (Eq. 3), f = -kappa rho T grad S
 *     - kappa_r rho c_p grad T; kappa_r may vary with radius as a quadratic
 *     in r (the solar case of Section 7.4), evaluated at the radius of each
 *     flux point given by the element map.
 *   - Rusanov wave speed max(|u_L.n| + c_L, |u_R.n| + c_R); one common flux
 *     per face point, shared by both sides.
 *   - BR1: gradients of the conserved variables from the flux-point values
 *     with the averaged interface solution at the ends, chain rule with the
 *     exact metrics at solution points, gradients interpolated to the flux
 *     points, viscous flux averaged at interfaces.
 *   - flux-point metrics in a conservative curl form adapted to the staggered
 *     SD lattice (free-stream preserving, watertight faces); solution-point
 *     metrics and |J| exact from the map.
 *   - walls: inviscid flux (0, p S, 0); viscous flux keeps only the normal
 *     traction; energy flux F_bottom at the inner wall, interior -f.n at the
 *     outer wall; BR1 wall state has the normal momentum removed at fixed p
 *     (outer wall: T = T_top when T_top > 0).
 */
#include "chorus_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static char g_err[256];
const char *ora_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* 1D operators                                                              */
/* ------------------------------------------------------------------------ */

/* Legendre polynomial of degree n on [0, 1] from P_{-1} = 0, P_0 = 1 and
 * P_n = (2n-1)/n (2x-1) P_{n-1} - (n-1)/n P_{n-2}. */
static double legendre01(int n, double x)
{
    double pm1 = 0.0, p = 1.0;
    for (int k = 1; k <= n; ++k) {
        double pn = (2.0 * k - 1.0) / k * (2.0 * x - 1.0) * p - (k - 1.0) / k * pm1;
        pm1 = p;
        p = pn;
    }
    return p;
}

/* h_s(x) = prod_{q != s} (x - X_q) / (X_s - X_q) over nodes X[0..n-1] */
static double lagrange(const double *X, int n, int s, double x)
{
    double v = 1.0;
    for (int q = 0; q < n; ++q)
        if (q != s)
            v *= (x - X[q]) / (X[s] - X[q]);
    return v;
}

/* derivative of the Lagrange basis polynomial by the product rule */
static double lagrange_d(const double *X, int n, int s, double x)
{
    double sum = 0.0;
    for (int r = 0; r < n; ++r) {
        if (r == s)
            continue;
        double t = 1.0 / (X[s] - X[r]);
        for (int q = 0; q < n; ++q)
            if (q != s && q != r)
                t *= (x - X[q]) / (X[s] - X[q]);
        sum += t;
    }
    return sum;
}

int ora_basis(int N, double *xs, double *xf, double *I, double *D, double *w)
{
    if (N < 2 || N > ORA_MAXN)
        return -1;
    /* solution points X_s = (1 - cos((2s-1) pi / (2N))) / 2, s = 1..N */
    for (int s = 1; s <= N; ++s)
        xs[s - 1] = 0.5 * (1.0 - cos((2.0 * s - 1.0) / (2.0 * N) * M_PI));
    /* flux points: 0, the N-1 roots of P_{N-1} (bisection), 1 */
    xf[0] = 0.0;
    xf[N] = 1.0;
    int found = 0;
    const int scan = 4000;
    double a = 0.0, fa = legendre01(N - 1, 0.0);
    for (int t = 1; t <= scan && found < N - 1; ++t) {
        double b = (double)t / scan, fb = legendre01(N - 1, b);
        if ((fa < 0.0) != (fb < 0.0)) {
            double lo = a, hi = b, flo = fa;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi), fm = legendre01(N - 1, mid);
                if (fm == 0.0) { lo = hi = mid; break; }
                if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else hi = mid;
                if (hi - lo < 1e-17) break;
            }
            xf[1 + found++] = 0.5 * (lo + hi);
        }
        a = b;
        fa = fb;
    }
    if (found != N - 1)
        return -2;
    for (int m = 0; m <= N; ++m)
        for (int s = 0; s < N; ++s)
            I[m * N + s] = lagrange(xs, N, s, xf[m]);
    for (int s = 0; s < N; ++s)
        for (int m = 0; m <= N; ++m)
            D[s * (N + 1) + m] = lagrange_d(xf, N + 1, m, xs[s]);
    /* w_s = int_0^1 h_s: expand h_s in monomials, integrate term by term */
    for (int s = 0; s < N; ++s) {
        double c[ORA_MAXN + 1] = {0};
        int deg = 0;
        c[0] = 1.0;
        for (int q = 0; q < N; ++q) {
            if (q == s)
                continue;
            double den = xs[s] - xs[q];
            double nc[ORA_MAXN + 1] = {0};
            for (int k = 0; k <= deg; ++k) {
                nc[k + 1] += c[k] / den;
                nc[k] -= c[k] * xs[q] / den;
            }
            ++deg;
            memcpy(c, nc, sizeof c);
        }
        double v = 0.0;
        for (int k = 0; k <= deg; ++k)
            v += c[k] / (k + 1.0);
        w[s] = v;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 20-node serendipity map on [0,1]^3                                        */
/* ------------------------------------------------------------------------ */
static const int LOC20[20][3] = {
    {0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {2, 2, 0}, {0, 0, 2}, {2, 0, 2}, {0, 2, 2}, {2, 2, 2},
    {1, 0, 0}, {1, 2, 0}, {1, 0, 2}, {1, 2, 2},
    {0, 1, 0}, {2, 1, 0}, {0, 1, 2}, {2, 1, 2},
    {0, 0, 1}, {2, 0, 1}, {0, 2, 1}, {2, 2, 1}};

/* x(r) and dx[c][i] = d x_c / d xi_i at reference point r in [0,1]^3 */
static void map_eval(const double nodes[20][3], const double r[3], double x[3], double dx[3][3])
{
    double a[3] = {2.0 * r[0] - 1.0, 2.0 * r[1] - 1.0, 2.0 * r[2] - 1.0};
    for (int c = 0; c < 3; ++c) {
        x[c] = 0.0;
        dx[c][0] = dx[c][1] = dx[c][2] = 0.0;
    }
    for (int n = 0; n < 20; ++n) {
        int p[3] = {LOC20[n][0] - 1, LOC20[n][1] - 1, LOC20[n][2] - 1};
        double Nn, dN[3];
        int zero_axis = -1;
        for (int t = 0; t < 3; ++t)
            if (p[t] == 0)
                zero_axis = t;
        if (zero_axis < 0) {
            /* corner: (1/8)(1+a p0)(1+b p1)(1+c p2)(a p0 + b p1 + c p2 - 2) */
            double f0 = 1.0 + a[0] * p[0], f1 = 1.0 + a[1] * p[1], f2 = 1.0 + a[2] * p[2];
            double s = a[0] * p[0] + a[1] * p[1] + a[2] * p[2] - 2.0;
            Nn = 0.125 * f0 * f1 * f2 * s;
            dN[0] = 0.125 * p[0] * f1 * f2 * (s + f0);
            dN[1] = 0.125 * p[1] * f0 * f2 * (s + f1);
            dN[2] = 0.125 * p[2] * f0 * f1 * (s + f2);
        } else {
            /* mid-edge along axis z: (1/4)(1 - a_z^2)(1 + a_u p_u)(1 + a_v p_v) */
            int z = zero_axis, u = (z + 1) % 3, v = (z + 2) % 3;
            double g = 1.0 - a[z] * a[z], fu = 1.0 + a[u] * p[u], fv = 1.0 + a[v] * p[v];
            Nn = 0.25 * g * fu * fv;
            dN[z] = 0.25 * (-2.0 * a[z]) * fu * fv;
            dN[u] = 0.25 * g * p[u] * fv;
            dN[v] = 0.25 * g * fu * p[v];
        }
        for (int c = 0; c < 3; ++c) {
            x[c] += Nn * nodes[n][c];
            for (int i = 0; i < 3; ++i)
                dx[c][i] += 2.0 * dN[i] * nodes[n][c]; /* d/dxi = 2 d/da */
        }
    }
}

/* ------------------------------------------------------------------------ */
/* mesh                                                                      */
/* ------------------------------------------------------------------------ */
struct ora_mesh {
    int N, np, nf2, nfl;    /* N, N^3, N^2, (N+1) N^2 */
    long E;
    double xs[ORA_MAXN], xf[ORA_MAXN + 1], I[(ORA_MAXN + 1) * ORA_MAXN],
        D[ORA_MAXN * (ORA_MAXN + 1)], w[ORA_MAXN];
    double *xsol;  /* [E][np][3] */
    double *jac;   /* [E][np] */
    double *met;   /* [E][np][3 d][3 c]  exact |J| grad xi_d */
    double *metf;  /* [E][3 d][nfl][3 c] curl-form |J| grad xi_d at d-flux points */
    double *rflux; /* [E][3 d][nfl] radius |x| at the d-flux points (from the map) */
    int *bc;       /* [E][6] */
    long *nbr_e;   /* [E][6] */
    int *nbr_f;    /* [E][6] */
    int *nbr_p;    /* [E][6][nf2] */
    /* residual work arrays */
    double *Qf, *Qs, *grad, *gradf, *Ft, *k1, *k2;
};

/* (i,j,k) of the point with index a along direction d and tangential
 * indices t1, t2 along the other two axes in increasing order */
static void dir_ijk(int d, int a, int t1, int t2, int ijk[3])
{
    if (d == 0) { ijk[0] = a; ijk[1] = t1; ijk[2] = t2; }
    else if (d == 1) { ijk[0] = t1; ijk[1] = a; ijk[2] = t2; }
    else { ijk[0] = t1; ijk[1] = t2; ijk[2] = a; }
}

static int sol_index(const ora_mesh *m, const int ijk[3])
{
    return ijk[0] + m->N * (ijk[1] + m->N * ijk[2]);
}

/* flux-point index within direction d: a along d (0..N), t1, t2 tangential */
static int fl_index(const ora_mesh *m, int a, int t1, int t2)
{
    return a + (m->N + 1) * (t1 + m->N * t2);
}

/* corner local index of face f's corner (c1, c2) (tangential axes in
 * increasing order) */
static int face_corner(int f, int c1, int c2)
{
    int d = f / 2, side = f % 2, ijk[3];
    dir_ijk(d, side, c1, c2, ijk);
    return ijk[0] + 2 * ijk[1] + 4 * ijk[2];
}

typedef struct { long key[4]; long e; int f; } face_rec;

static int cmp_long(const void *a, const void *b)
{
    long x = *(const long *)a, y = *(const long *)b;
    return (x > y) - (x < y);
}

static int cmp_face(const void *a, const void *b)
{
    const face_rec *x = a, *y = b;
    for (int t = 0; t < 4; ++t)
        if (x->key[t] != y->key[t])
            return (x->key[t] > y->key[t]) - (x->key[t] < y->key[t]);
    if (x->e != y->e)
        return (x->e > y->e) - (x->e < y->e);
    return x->f - y->f;
}

/* weight of face point (s, t) on the corner whose id is cid */
static double corner_weight(const long ids[2][2], long cid, double s, double t)
{
    double wsum = 0.0;
    for (int c2 = 0; c2 < 2; ++c2)
        for (int c1 = 0; c1 < 2; ++c1)
            if (ids[c1][c2] == cid)
                wsum += (c1 ? s : 1.0 - s) * (c2 ? t : 1.0 - t);
    return wsum;
}

void ora_mesh_free(ora_mesh *m)
{
    if (!m)
        return;
    free(m->xsol); free(m->jac); free(m->met); free(m->metf); free(m->rflux); free(m->bc);
    free(m->nbr_e); free(m->nbr_f); free(m->nbr_p);
    free(m->Qf); free(m->Qs); free(m->grad); free(m->gradf); free(m->Ft);
    free(m->k1); free(m->k2);
    free(m);
}

ora_mesh *ora_mesh_new(int N, long n_nodes, const double *xyz, long n_elems,
                       const long *elem20, const int *face_bc, const long *match_id)
{
    g_err[0] = 0;
    ora_mesh *m = calloc(1, sizeof *m);
    if (!m)
        return NULL;
    if (ora_basis(N, m->xs, m->xf, m->I, m->D, m->w) != 0) {
        snprintf(g_err, sizeof g_err, "unsupported order %d", N);
        free(m);
        return NULL;
    }
    m->N = N;
    m->np = N * N * N;
    m->nf2 = N * N;
    m->nfl = (N + 1) * N * N;
    m->E = n_elems;
    long E = n_elems;
    m->xsol = malloc(sizeof(double) * E * m->np * 3);
    m->jac = malloc(sizeof(double) * E * m->np);
    m->met = malloc(sizeof(double) * E * m->np * 9);
    m->metf = malloc(sizeof(double) * E * 3 * m->nfl * 3);
    m->rflux = malloc(sizeof(double) * E * 3 * m->nfl);
    m->bc = malloc(sizeof(int) * E * 6);
    m->nbr_e = malloc(sizeof(long) * E * 6);
    m->nbr_f = malloc(sizeof(int) * E * 6);
    m->nbr_p = malloc(sizeof(int) * E * 6 * m->nf2);
    for (long e = 0; e < E; ++e) {
        for (int n = 0; n < 20; ++n) {
            long id = elem20[e * 20 + n];
            if (id < 0 || id >= n_nodes) {
                snprintf(g_err, sizeof g_err, "element %ld node %d out of range", e, n);
                ora_mesh_free(m);
                return NULL;
            }
        }
    }

    /* ---- faces: match element faces by their sorted corner ids ---- */
    face_rec *recs = malloc(sizeof(face_rec) * E * 6);
    long nrec = 0;
    for (long e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            m->bc[e * 6 + f] = face_bc[e * 6 + f];
            m->nbr_e[e * 6 + f] = -1;
            m->nbr_f[e * 6 + f] = -1;
            for (int p = 0; p < m->nf2; ++p)
                m->nbr_p[(e * 6 + f) * m->nf2 + p] = -1;
            if (face_bc[e * 6 + f] >= 0)
                continue;
            face_rec *r = &recs[nrec++];
            int t = 0;
            for (int c2 = 0; c2 < 2; ++c2)
                for (int c1 = 0; c1 < 2; ++c1) {
                    long node = elem20[e * 20 + face_corner(f, c1, c2)];
                    r->key[t++] = match_id ? match_id[node] : node;
                }
            qsort(r->key, 4, sizeof(long), cmp_long);
            r->e = e;
            r->f = f;
        }
    qsort(recs, nrec, sizeof(face_rec), cmp_face);
    for (long t = 0; t < nrec;) {
        if (t + 1 >= nrec || memcmp(recs[t].key, recs[t + 1].key, sizeof recs[t].key) != 0
            || (t + 2 < nrec && memcmp(recs[t].key, recs[t + 2].key, sizeof recs[t].key) == 0)) {
            snprintf(g_err, sizeof g_err, "unmatched interior face (element %ld face %d)",
                     recs[t].e, recs[t].f);
            free(recs);
            ora_mesh_free(m);
            return NULL;
        }
        for (int side = 0; side < 2; ++side) {
            face_rec *a = &recs[t + side], *b = &recs[t + 1 - side];
            m->nbr_e[a->e * 6 + a->f] = b->e;
            m->nbr_f[a->e * 6 + a->f] = b->f;
        }
        t += 2;
    }
    free(recs);
    /* face points: brute-force match by bilinear weights on the shared
     * corner ids */
    for (long e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            long e2 = m->nbr_e[e * 6 + f];
            if (e2 < 0)
                continue;
            int f2 = m->nbr_f[e * 6 + f];
            long ida[2][2], idb[2][2];
            for (int c2 = 0; c2 < 2; ++c2)
                for (int c1 = 0; c1 < 2; ++c1) {
                    long na = elem20[e * 20 + face_corner(f, c1, c2)];
                    long nb = elem20[e2 * 20 + face_corner(f2, c1, c2)];
                    ida[c1][c2] = match_id ? match_id[na] : na;
                    idb[c1][c2] = match_id ? match_id[nb] : nb;
                }
            for (int t2 = 0; t2 < N; ++t2)
                for (int t1 = 0; t1 < N; ++t1) {
                    double s = m->xs[t1], tt = m->xs[t2];
                    int hit = -1;
                    for (int u2 = 0; u2 < N && hit < 0; ++u2)
                        for (int u1 = 0; u1 < N; ++u1) {
                            double s2 = m->xs[u1], ttt = m->xs[u2];
                            int ok = 1;
                            for (int c2 = 0; c2 < 2 && ok; ++c2)
                                for (int c1 = 0; c1 < 2; ++c1) {
                                    long cid = ida[c1][c2];
                                    double wa = corner_weight(ida, cid, s, tt);
                                    double wb = corner_weight(idb, cid, s2, ttt);
                                    if (fabs(wa - wb) > 1e-12) { ok = 0; break; }
                                }
                            if (ok) { hit = u1 + N * u2; break; }
                        }
                    if (hit < 0) {
                        snprintf(g_err, sizeof g_err, "face point unmatched (element %ld face %d)", e, f);
                        ora_mesh_free(m);
                        return NULL;
                    }
                    m->nbr_p[(e * 6 + f) * m->nf2 + t1 + N * t2] = hit;
                }
        }

    /* ---- geometry ---- */
    int L = N + 1, L3 = L * L * L;
    double *W = malloc(sizeof(double) * 9 * L3); /* W[n][i][lattice] */
    for (long e = 0; e < E; ++e) {
        double nodes[20][3];
        for (int n = 0; n < 20; ++n)
            for (int c = 0; c < 3; ++c)
                nodes[n][c] = xyz[elem20[e * 20 + n] * 3 + c];
        /* solution points: x, |J|, |J| grad xi_d = dx/dxi_d1 x dx/dxi_d2 */
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    int p = i + N * (j + N * k);
                    double r[3] = {m->xs[i], m->xs[j], m->xs[k]}, x[3], dx[3][3];
                    map_eval(nodes, r, x, dx);
                    for (int c = 0; c < 3; ++c)
                        m->xsol[(e * m->np + p) * 3 + c] = x[c];
                    double det = dx[0][0] * (dx[1][1] * dx[2][2] - dx[1][2] * dx[2][1])
                               - dx[0][1] * (dx[1][0] * dx[2][2] - dx[1][2] * dx[2][0])
                               + dx[0][2] * (dx[1][0] * dx[2][1] - dx[1][1] * dx[2][0]);
                    if (!(det > 0.0)) {
                        snprintf(g_err, sizeof g_err, "non-positive Jacobian in element %ld", e);
                        free(W);
                        ora_mesh_free(m);
                        return NULL;
                    }
                    m->jac[e * m->np + p] = det;
                    for (int d = 0; d < 3; ++d) {
                        int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
                        double *o = &m->met[((e * m->np + p) * 3 + d) * 3];
                        o[0] = dx[1][d1] * dx[2][d2] - dx[2][d1] * dx[1][d2];
                        o[1] = dx[2][d1] * dx[0][d2] - dx[0][d1] * dx[2][d2];
                        o[2] = dx[0][d1] * dx[1][d2] - dx[1][d1] * dx[0][d2];
                    }
                }
        /* radius at the d-flux points: reference coordinate xf[a] along d,
         * solution-point coordinates along the other two axes */
        for (int d = 0; d < 3; ++d)
            for (int t2 = 0; t2 < N; ++t2)
                for (int t1 = 0; t1 < N; ++t1)
                    for (int a = 0; a <= N; ++a) {
                        int idx[3];
                        dir_ijk(d, a, t1, t2, idx);
                        double r[3], x[3], dx[3][3];
                        for (int t = 0; t < 3; ++t)
                            r[t] = (t == d) ? m->xf[idx[t]] : m->xs[idx[t]];
                        map_eval(nodes, r, x, dx);
                        m->rflux[(e * 3 + d) * m->nfl + fl_index(m, a, t1, t2)]
                            = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                    }
        /* curl form: W^(n)_i = x_l d x_m / d xi_i, (n, m, l) cyclic, sampled
         * on the lattice with solution points along i and flux points along
         * the other two axes */
        for (int i = 0; i < 3; ++i)
            for (int a2 = 0; a2 < L; ++a2)
                for (int a1 = 0; a1 < L; ++a1)
                    for (int a0 = 0; a0 < L; ++a0) {
                        int idx[3] = {a0, a1, a2};
                        if (idx[i] >= N)
                            continue;
                        double r[3], x[3], dx[3][3];
                        for (int t = 0; t < 3; ++t)
                            r[t] = (t == i) ? m->xs[idx[t]] : m->xf[idx[t]];
                        map_eval(nodes, r, x, dx);
                        for (int n = 0; n < 3; ++n) {
                            int mm = (n + 1) % 3, l = (n + 2) % 3;
                            W[(n * 3 + i) * L3 + a0 + L * (a1 + L * a2)] = x[l] * dx[mm][i];
                        }
                    }
        /* |J| grad xi_d at d-flux points = -(curl_xi W^(n))_d */
        for (int d = 0; d < 3; ++d) {
            int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
            for (int t2 = 0; t2 < N; ++t2)
                for (int t1 = 0; t1 < N; ++t1)
                    for (int a = 0; a <= N; ++a) {
                        int idx[3];
                        dir_ijk(d, a, t1, t2, idx);
                        for (int n = 0; n < 3; ++n) {
                            double term1 = 0.0, term2 = 0.0;
                            for (int q = 0; q <= N; ++q) {
                                int j1[3] = {idx[0], idx[1], idx[2]};
                                j1[d1] = q;
                                term1 += m->D[idx[d1] * (N + 1) + q]
                                         * W[(n * 3 + d2) * L3 + j1[0] + L * (j1[1] + L * j1[2])];
                                int j2[3] = {idx[0], idx[1], idx[2]};
                                j2[d2] = q;
                                term2 += m->D[idx[d2] * (N + 1) + q]
                                         * W[(n * 3 + d1) * L3 + j2[0] + L * (j2[1] + L * j2[2])];
                            }
                            m->metf[((e * 3 + d) * m->nfl + fl_index(m, a, t1, t2)) * 3 + n]
                                = -(term1 - term2);
                        }
                    }
        }
    }
    free(W);

    m->Qf = malloc(sizeof(double) * 3 * E * 5 * m->nfl);
    m->Qs = malloc(sizeof(double) * E * 6 * 5 * m->nf2);
    m->grad = malloc(sizeof(double) * E * 15 * m->np);
    m->gradf = malloc(sizeof(double) * 3 * E * 15 * m->nfl);
    m->Ft = malloc(sizeof(double) * 3 * E * 5 * m->nfl);
    m->k1 = malloc(sizeof(double) * 5 * E * m->np);
    m->k2 = malloc(sizeof(double) * 5 * E * m->np);
    if (!m->Qf || !m->Qs || !m->grad || !m->gradf || !m->Ft || !m->k1 || !m->k2) {
        snprintf(g_err, sizeof g_err, "out of memory");
        ora_mesh_free(m);
        return NULL;
    }
    return m;
}

void ora_solpts(const ora_mesh *m, double *xyz, double *wJ)
{
    int N = m->N;
    long n = m->E * m->np;
    for (long e = 0; e < m->E; ++e)
        for (int p = 0; p < m->np; ++p) {
            long g = e * m->np + p;
            for (int c = 0; c < 3; ++c)
                xyz[c * n + g] = m->xsol[g * 3 + c];
            int i = p % N, j = (p / N) % N, k = p / (N * N);
            wJ[g] = m->w[i] * m->w[j] * m->w[k] * m->jac[g];
        }
}

void ora_geometry(const ora_mesh *m, double *jac, double *met_sol, double *met_flux)
{
    long n = m->E * m->np;
    if (jac) memcpy(jac, m->jac, sizeof(double) * n);
    if (met_sol) memcpy(met_sol, m->met, sizeof(double) * n * 9);
    if (met_flux) memcpy(met_flux, m->metf, sizeof(double) * m->E * 3 * m->nfl * 3);
}

void ora_faces(const ora_mesh *m, long *nbr_e, int *nbr_f, int *nbr_p)
{
    memcpy(nbr_e, m->nbr_e, sizeof(long) * m->E * 6);
    memcpy(nbr_f, m->nbr_f, sizeof(int) * m->E * 6);
    memcpy(nbr_p, m->nbr_p, sizeof(int) * m->E * 6 * m->nf2);
}

/* ------------------------------------------------------------------------ */
/* physical fluxes (Section 2)                                               */
/* ------------------------------------------------------------------------ */
static double pressure(const ora_phys *ph, const double q[5])
{
    return (ph->gamma - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
}

/* (F_inv, G_inv, H_inv) . S for a (not necessarily unit) vector S */
static void inviscid_flux(const ora_phys *ph, const double q[5], const double S[3], double out[5])
{
    double rho = q[0], u[3] = {q[1] / rho, q[2] / rho, q[3] / rho};
    double p = pressure(ph, q);
    double un = u[0] * S[0] + u[1] * S[1] + u[2] * S[2];
    out[0] = rho * un;
    out[1] = q[1] * un + p * S[0];
    out[2] = q[2] * un + p * S[1];
    out[3] = q[3] * un + p * S[2];
    out[4] = (q[4] + p) * un;
}

/* primitive gradients from conserved gradients g[v][c] = d Q_v / d x_c */
typedef struct { double u[3], du[3][3], rho, p, T, dS[3], dT[3]; } prim_grad;

static void primitive_gradients(const ora_phys *ph, const double q[5], const double g[5][3], prim_grad *o)
{
    double gam = ph->gamma, R = ph->R_gas, cp = gam * R / (gam - 1.0);
    o->rho = q[0];
    for (int a = 0; a < 3; ++a)
        o->u[a] = q[1 + a] / q[0];
    o->p = pressure(ph, q);
    o->T = o->p / (o->rho * R);
    double uu = o->u[0] * o->u[0] + o->u[1] * o->u[1] + o->u[2] * o->u[2];
    for (int c = 0; c < 3; ++c) {
        for (int a = 0; a < 3; ++a)
            o->du[a][c] = (g[1 + a][c] - o->u[a] * g[0][c]) / o->rho;
        double dp = (gam - 1.0) * (g[4][c] - (o->u[0] * g[1][c] + o->u[1] * g[2][c] + o->u[2] * g[3][c])
                                   + 0.5 * uu * g[0][c]);
        /* S = c_p ln(p^(1/gamma) / rho) */
        o->dS[c] = cp * (dp / (gam * o->p) - g[0][c] / o->rho);
        /* T = p / (rho R) */
        o->dT[c] = (dp - R * o->T * g[0][c]) / (o->rho * R);
    }
}

/* Newtonian stress with mu = rho nu (Section 2) */
static void stress(const ora_phys *ph, const prim_grad *pg, double tau[3][3])
{
    double mu = pg->rho * ph->nu;
    double div = pg->du[0][0] + pg->du[1][1] + pg->du[2][2];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            tau[a][b] = mu * (pg->du[a][b] + pg->du[b][a]) - (a == b ? 2.0 / 3.0 * mu * div : 0.0);
}

/* radiative diffusivity at radius r: the constant, or the quadratic in r
 * of the solar case (Section 7.4) */
static double kappa_r_at(const ora_phys *ph, double r)
{
    return ph->kappa_r + ph->kappa_r1 * r + ph->kappa_r2 * r * r;
}

/* (F_v, G_v, H_v) . S, energy component u.tau.S - f.S; kr = kappa_r at the
 * point */
static void viscous_flux(const ora_phys *ph, const double q[5], const double g[5][3], const double S[3],
                         double kr, double out[5])
{
    prim_grad pg;
    primitive_gradients(ph, q, g, &pg);
    double tau[3][3];
    stress(ph, &pg, tau);
    double cp = ph->gamma * ph->R_gas / (ph->gamma - 1.0);
    double tS[3];
    for (int a = 0; a < 3; ++a)
        tS[a] = tau[a][0] * S[0] + tau[a][1] * S[1] + tau[a][2] * S[2];
    double dSS = pg.dS[0] * S[0] + pg.dS[1] * S[1] + pg.dS[2] * S[2];
    double dTS = pg.dT[0] * S[0] + pg.dT[1] * S[1] + pg.dT[2] * S[2];
    out[0] = 0.0;
    out[1] = tS[0];
    out[2] = tS[1];
    out[3] = tS[2];
    out[4] = pg.u[0] * tS[0] + pg.u[1] * tS[1] + pg.u[2] * tS[2]
           + ph->kappa * pg.rho * pg.T * dSS + kr * pg.rho * cp * dTS;
}

/* Rusanov common inviscid flux along S (outward from the L side) */
static void rusanov(const ora_phys *ph, const double qL[5], const double qR[5], const double S[3],
                    double out[5])
{
    double A = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    double n[3] = {S[0] / A, S[1] / A, S[2] / A};
    double fL[5], fR[5];
    inviscid_flux(ph, qL, S, fL);
    inviscid_flux(ph, qR, S, fR);
    double unL = (qL[1] * n[0] + qL[2] * n[1] + qL[3] * n[2]) / qL[0];
    double unR = (qR[1] * n[0] + qR[2] * n[1] + qR[3] * n[2]) / qR[0];
    double cL = sqrt(ph->gamma * pressure(ph, qL) / qL[0]);
    double cR = sqrt(ph->gamma * pressure(ph, qR) / qR[0]);
    double lam = fmax(fabs(unL) + cL, fabs(unR) + cR);
    for (int v = 0; v < 5; ++v)
        out[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * lam * A * (qR[v] - qL[v]);
}

/* BR1 wall state: normal momentum removed, pressure kept (outer wall with
 * T_top > 0: temperature set to T_top) */
static void wall_state(const ora_phys *ph, const double q[5], const double n[3], int outer, double qb[5])
{
    double mn = q[1] * n[0] + q[2] * n[1] + q[3] * n[2];
    double p = pressure(ph, q);
    if (outer && ph->T_top > 0.0)
        p = q[0] * ph->R_gas * ph->T_top;
    qb[0] = q[0];
    for (int a = 0; a < 3; ++a)
        qb[1 + a] = q[1 + a] - mn * n[a];
    qb[4] = p / (ph->gamma - 1.0) + 0.5 * (qb[1] * qb[1] + qb[2] * qb[2] + qb[3] * qb[3]) / qb[0];
}

/* ------------------------------------------------------------------------ */
/* residual                                                                  */
/* ------------------------------------------------------------------------ */
#define QF(d, e, v, f) Qf[(((long)(d) * E + (e)) * 5 + (v)) * nfl + (f)]
#define QS(e, fc, v, p) Qs[(((e) * 6 + (fc)) * 5 + (v)) * nf2 + (p)]
#define GR(e, v, c, p) grad[(((e) * 5 + (v)) * 3 + (c)) * np + (p)]
#define GF(d, e, v, c, f) gradf[((((long)(d) * E + (e)) * 5 + (v)) * 3 + (c)) * nfl + (f)]
#define FT(d, e, v, f) Ft[(((long)(d) * E + (e)) * 5 + (v)) * nfl + (f)]
#define QIN(v, e, p) Q[((long)(v) * E + (e)) * np + (p)]

/* steps 1-3 of the residual: flux-point values, common interface solution
 * and the BR1 gradients of the conserved variables at the solution points
 * (left in m->Qf, m->Qs, m->grad) */
static void interface_and_gradients(const ora_mesh *m, const ora_phys *ph, const double *Q)
{
    const int N = m->N, np = m->np, nf2 = m->nf2, nfl = m->nfl;
    const long E = m->E;
    double *Qf = m->Qf, *Qs = m->Qs, *grad = m->grad;

    /* step 1: Q at the flux points of each direction (interpolation along
     * the line through the flux point) */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e)
        for (int d = 0; d < 3; ++d)
            for (int t2 = 0; t2 < N; ++t2)
                for (int t1 = 0; t1 < N; ++t1)
                    for (int a = 0; a <= N; ++a)
                        for (int v = 0; v < 5; ++v) {
                            double s = 0.0;
                            for (int b = 0; b < N; ++b) {
                                int ijk[3];
                                dir_ijk(d, b, t1, t2, ijk);
                                s += m->I[a * N + b] * QIN(v, e, sol_index(m, ijk));
                            }
                            QF(d, e, v, fl_index(m, a, t1, t2)) = s;
                        }

    /* step 2: common interface solution (BR1 average / wall state) */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e)
        for (int fc = 0; fc < 6; ++fc) {
            int d = fc / 2, side = fc % 2, aend = side ? N : 0;
            for (int t2 = 0; t2 < N; ++t2)
                for (int t1 = 0; t1 < N; ++t1) {
                    int p = t1 + N * t2, fi = fl_index(m, aend, t1, t2);
                    double own[5], qs[5];
                    for (int v = 0; v < 5; ++v)
                        own[v] = QF(d, e, v, fi);
                    int bcv = m->bc[e * 6 + fc];
                    if (bcv < 0) {
                        long e2 = m->nbr_e[e * 6 + fc];
                        int f2 = m->nbr_f[e * 6 + fc], p2 = m->nbr_p[(e * 6 + fc) * nf2 + p];
                        int d2 = f2 / 2, a2 = (f2 % 2) ? N : 0;
                        int fi2 = fl_index(m, a2, p2 % N, p2 / N);
                        for (int v = 0; v < 5; ++v)
                            qs[v] = 0.5 * (own[v] + QF(d2, e2, v, fi2));
                    } else if (bcv == 1 || bcv == 2) {
                        const double *S = &m->metf[((e * 3 + d) * nfl + fi) * 3];
                        double sg = side ? 1.0 : -1.0;
                        double A = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
                        double n[3] = {sg * S[0] / A, sg * S[1] / A, sg * S[2] / A};
                        wall_state(ph, own, n, bcv == 2, qs);
                    } else {
                        for (int v = 0; v < 5; ++v)
                            qs[v] = 0.5 * (own[v] + ph->bc_state[v]);
                    }
                    for (int v = 0; v < 5; ++v)
                        QS(e, fc, v, p) = qs[v];
                }
        }

    /* step 3: gradients at solution points: derivative of the flux-point
     * polynomial (common values at the ends), then the chain rule
     * grad_x Q = (1/|J|) sum_d (|J| grad xi_d) dQ/dxi_d */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e)
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    int ijk[3] = {i, j, k}, p = sol_index(m, ijk);
                    double dq[3][5];
                    for (int d = 0; d < 3; ++d) {
                        int a = ijk[d], t1, t2;
                        if (d == 0) { t1 = j; t2 = k; } else if (d == 1) { t1 = i; t2 = k; } else { t1 = i; t2 = j; }
                        for (int v = 0; v < 5; ++v) {
                            double s = 0.0;
                            for (int mm = 0; mm <= N; ++mm) {
                                double qv;
                                if (mm == 0) qv = QS(e, 2 * d, v, t1 + N * t2);
                                else if (mm == N) qv = QS(e, 2 * d + 1, v, t1 + N * t2);
                                else qv = QF(d, e, v, fl_index(m, mm, t1, t2));
                                s += m->D[a * (N + 1) + mm] * qv;
                            }
                            dq[d][v] = s;
                        }
                    }
                    double J = m->jac[e * np + p];
                    for (int v = 0; v < 5; ++v)
                        for (int c = 0; c < 3; ++c) {
                            double s = 0.0;
                            for (int d = 0; d < 3; ++d)
                                s += m->met[((e * np + p) * 3 + d) * 3 + c] * dq[d][v];
                            GR(e, v, c, p) = s / J;
                        }
                }

}

/* Gradients of the conserved variables at the solution points, the BR1
 * values the viscous flux uses (Section 3): out[v*3+c][E][N^3] = dQ_v/dx_c. */
void ora_gradients(const ora_mesh *m, const ora_phys *ph, const double *Q, double *out)
{
    const int np = m->np;
    const long E = m->E;
    const double *grad = m->grad;
    interface_and_gradients(m, ph, Q);
    for (long e = 0; e < E; ++e)
        for (int v = 0; v < 5; ++v)
            for (int c = 0; c < 3; ++c)
                for (int p = 0; p < np; ++p)
                    out[((long)(v * 3 + c) * E + e) * np + p] = GR(e, v, c, p);
}

void ora_residual(const ora_mesh *m, const ora_phys *ph, const double *Q, double *dQdt)
{
    ora_residual_sgs(m, ph, Q, NULL, dQdt);
}

/* Residual with an additional flux: sgs[v*3+c][E][N^3] (Cartesian
 * component c of a flux of variable v at the solution points, e.g. a
 * learned subgrid-scale flux) enters the total flux F_inv - F_v + sgs.  It is
 * interpolated to the flux points along each line like the gradients,
 * averaged between the two sides at interior interfaces and left out at
 * wall and far-field faces (no subgrid transport through a boundary). */
void ora_residual_sgs(const ora_mesh *m, const ora_phys *ph, const double *Q, const double *sgs,
                      double *dQdt)
{
    const int N = m->N, np = m->np, nf2 = m->nf2, nfl = m->nfl;
    const long E = m->E;
    double *Qf = m->Qf, *grad = m->grad, *gradf = m->gradf, *Ft = m->Ft;
    double *sgsf = NULL;
#define SF(d, e, v, c, f) sgsf[((((long)(d) * E + (e)) * 5 + (v)) * 3 + (c)) * nfl + (f)]

    interface_and_gradients(m, ph, Q);

    /* step 4b: the additional flux at the flux points */
    if (sgs) {
        sgsf = malloc(sizeof(double) * 3 * E * 15 * nfl);
        if (!sgsf)
            abort();
#pragma omp parallel for schedule(static)
        for (long e = 0; e < E; ++e)
            for (int d = 0; d < 3; ++d)
                for (int t2 = 0; t2 < N; ++t2)
                    for (int t1 = 0; t1 < N; ++t1)
                        for (int a = 0; a <= N; ++a)
                            for (int v = 0; v < 5; ++v)
                                for (int c = 0; c < 3; ++c) {
                                    double s = 0.0;
                                    for (int b = 0; b < N; ++b) {
                                        int ijk[3];
                                        dir_ijk(d, b, t1, t2, ijk);
                                        s += m->I[a * N + b] * sgs[((long)(v * 3 + c) * E + e) * np + sol_index(m, ijk)];
                                    }
                                    SF(d, e, v, c, fl_index(m, a, t1, t2)) = s;
                                }
    }

    /* step 4: gradients interpolated to the flux points */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e)
        for (int d = 0; d < 3; ++d)
            for (int t2 = 0; t2 < N; ++t2)
                for (int t1 = 0; t1 < N; ++t1)
                    for (int a = 0; a <= N; ++a)
                        for (int v = 0; v < 5; ++v)
                            for (int c = 0; c < 3; ++c) {
                                double s = 0.0;
                                for (int b = 0; b < N; ++b) {
                                    int ijk[3];
                                    dir_ijk(d, b, t1, t2, ijk);
                                    s += m->I[a * N + b] * GR(e, v, c, sol_index(m, ijk));
                                }
                                GF(d, e, v, c, fl_index(m, a, t1, t2)) = s;
                            }

    /* step 5: transformed fluxes at interior flux points,
     * F~ = (|J| grad xi_d) . (F_inv - F_v) */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e)
        for (int d = 0; d < 3; ++d)
            for (int t2 = 0; t2 < N; ++t2)
                for (int t1 = 0; t1 < N; ++t1)
                    for (int a = 1; a < N; ++a) {
                        int fi = fl_index(m, a, t1, t2);
                        double q[5], g[5][3], fi_[5], fv[5];
                        for (int v = 0; v < 5; ++v) {
                            q[v] = QF(d, e, v, fi);
                            for (int c = 0; c < 3; ++c)
                                g[v][c] = GF(d, e, v, c, fi);
                        }
                        const double *S = &m->metf[((e * 3 + d) * nfl + fi) * 3];
                        inviscid_flux(ph, q, S, fi_);
                        viscous_flux(ph, q, g, S, kappa_r_at(ph, m->rflux[(e * 3 + d) * nfl + fi]), fv);
                        for (int v = 0; v < 5; ++v) {
                            FT(d, e, v, fi) = fi_[v] - fv[v];
                            if (sgsf)
                                for (int c = 0; c < 3; ++c)
                                    FT(d, e, v, fi) += SF(d, e, v, c, fi) * S[c];
                        }
                    }

    /* step 6: common fluxes at the interface points.  Each interior face is
     * evaluated once, by the side with the smaller (element, face) pair,
     * with its area vector; the other side receives the negated value. */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e)
        for (int fc = 0; fc < 6; ++fc) {
            int bcv = m->bc[e * 6 + fc];
            long e2 = m->nbr_e[e * 6 + fc];
            int f2 = m->nbr_f[e * 6 + fc];
            if (bcv < 0 && (e2 * 6 + f2) < (e * 6 + fc))
                continue; /* evaluated by the other side */
            int d = fc / 2, side = fc % 2, aend = side ? N : 0;
            double sg = side ? 1.0 : -1.0;
            for (int t2 = 0; t2 < N; ++t2)
                for (int t1 = 0; t1 < N; ++t1) {
                    int p = t1 + N * t2, fi = fl_index(m, aend, t1, t2);
                    const double *Sd = &m->metf[((e * 3 + d) * nfl + fi) * 3];
                    double S[3] = {sg * Sd[0], sg * Sd[1], sg * Sd[2]};
                    double A = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
                    double qL[5], gL[5][3], phi[5];
                    for (int v = 0; v < 5; ++v) {
                        qL[v] = QF(d, e, v, fi);
                        for (int c = 0; c < 3; ++c)
                            gL[v][c] = GF(d, e, v, c, fi);
                    }
                    if (bcv < 0) {
                        int p2 = m->nbr_p[(e * 6 + fc) * nf2 + p];
                        int d2 = f2 / 2, a2 = (f2 % 2) ? N : 0;
                        int fi2 = fl_index(m, a2, p2 % N, p2 / N);
                        double qR[5], gR[5][3], fvL[5], fvR[5];
                        for (int v = 0; v < 5; ++v) {
                            qR[v] = QF(d2, e2, v, fi2);
                            for (int c = 0; c < 3; ++c)
                                gR[v][c] = GF(d2, e2, v, c, fi2);
                        }
                        rusanov(ph, qL, qR, S, phi);
                        viscous_flux(ph, qL, gL, S, kappa_r_at(ph, m->rflux[(e * 3 + d) * nfl + fi]), fvL);
                        viscous_flux(ph, qR, gR, S, kappa_r_at(ph, m->rflux[((long)e2 * 3 + d2) * nfl + fi2]), fvR);
                        for (int v = 0; v < 5; ++v)
                            phi[v] -= 0.5 * (fvL[v] + fvR[v]);
                        if (sgsf)
                            for (int v = 0; v < 5; ++v)
                                for (int c = 0; c < 3; ++c)
                                    phi[v] += 0.5 * (SF(d, e, v, c, fi) + SF(d2, e2, v, c, fi2)) * S[c];
                        double sg2 = (f2 % 2) ? 1.0 : -1.0;
                        for (int v = 0; v < 5; ++v)
                            FT(d2, e2, v, fi2) = sg2 * (-phi[v]);
                    } else if (bcv == 1 || bcv == 2) {
                        double n[3] = {S[0] / A, S[1] / A, S[2] / A};
                        prim_grad pg;
                        primitive_gradients(ph, qL, gL, &pg);
                        double tau[3][3];
                        stress(ph, &pg, tau);
                        double tnn = 0.0;
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b)
                                tnn += n[a] * tau[a][b] * n[b];
                        double p_in = pressure(ph, qL);
                        double energy_v;
                        if (bcv == 1) {
                            energy_v = ph->F_bottom * A;
                        } else {
                            double cp = ph->gamma * ph->R_gas / (ph->gamma - 1.0);
                            double dSS = pg.dS[0] * S[0] + pg.dS[1] * S[1] + pg.dS[2] * S[2];
                            double dTS = pg.dT[0] * S[0] + pg.dT[1] * S[1] + pg.dT[2] * S[2];
                            energy_v = ph->kappa * pg.rho * pg.T * dSS
                                     + kappa_r_at(ph, m->rflux[(e * 3 + d) * nfl + fi]) * pg.rho * cp * dTS;
                        }
                        phi[0] = 0.0;
                        for (int a = 0; a < 3; ++a)
                            phi[1 + a] = p_in * S[a] - tnn * S[a];
                        phi[4] = -energy_v;
                    } else {
                        double fvL[5];
                        rusanov(ph, qL, ph->bc_state, S, phi);
                        viscous_flux(ph, qL, gL, S, kappa_r_at(ph, m->rflux[(e * 3 + d) * nfl + fi]), fvL);
                        for (int v = 0; v < 5; ++v)
                            phi[v] -= 0.5 * fvL[v];
                    }
                    for (int v = 0; v < 5; ++v)
                        FT(d, e, v, fi) = sg * phi[v];
                }
        }

    /* steps 7-8: divergence of the flux polynomials and the source,
     * dQ/dt = -(dF~/dxi + dG~/deta + dH~/dzeta) / |J| - M */
#pragma omp parallel for schedule(static)
    for (long e = 0; e < E; ++e)
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    int ijk[3] = {i, j, k}, p = sol_index(m, ijk);
                    double div[5] = {0, 0, 0, 0, 0};
                    for (int d = 0; d < 3; ++d) {
                        int a = ijk[d], t1, t2;
                        if (d == 0) { t1 = j; t2 = k; } else if (d == 1) { t1 = i; t2 = k; } else { t1 = i; t2 = j; }
                        for (int v = 0; v < 5; ++v)
                            for (int mm = 0; mm <= N; ++mm)
                                div[v] += m->D[a * (N + 1) + mm] * FT(d, e, v, fl_index(m, mm, t1, t2));
                    }
                    double J = m->jac[e * np + p];
                    const double *x = &m->xsol[(e * np + p) * 3];
                    double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                    double gf = ph->GM / (r * r * r);
                    double g[3] = {gf * x[0], gf * x[1], gf * x[2]};
                    double rho = QIN(0, e, p), mx = QIN(1, e, p), my = QIN(2, e, p), mz = QIN(3, e, p);
                    double M[5];
                    M[0] = 0.0;
                    M[1] = rho * g[0] - 2.0 * ph->omega * my;
                    M[2] = rho * g[1] + 2.0 * ph->omega * mx;
                    M[3] = rho * g[2];
                    M[4] = mx * g[0] + my * g[1] + mz * g[2];
                    for (int v = 0; v < 5; ++v)
                        dQdt[((long)v * E + e) * np + p] = -div[v] / J - M[v];
                }
    free(sgsf);
#undef SF
}
#undef QF
#undef QS
#undef GR
#undef GF
#undef FT
#undef QIN

/* SSP-RK3 (Shu-Osher form) */
void ora_rk3(const ora_mesh *m, const ora_phys *ph, double *Q, double dt, int nsteps)
{
    long n = 5 * m->E * m->np;
    double *Q1 = m->k1, *R = m->k2;
    for (int st = 0; st < nsteps; ++st) {
        ora_residual(m, ph, Q, R);
        for (long t = 0; t < n; ++t)
            Q1[t] = Q[t] + dt * R[t];
        ora_residual(m, ph, Q1, R);
        for (long t = 0; t < n; ++t)
            Q1[t] = 0.75 * Q[t] + 0.25 * (Q1[t] + dt * R[t]);
        ora_residual(m, ph, Q1, R);
        for (long t = 0; t < n; ++t)
            Q[t] = Q[t] / 3.0 + 2.0 / 3.0 * (Q1[t] + dt * R[t]);
    }
}

/* Five-stage fourth-order SSP Runge-Kutta, SSPRK(5,4) of Spiteri & Ruuth
 * (2002), in Shu-Osher form u_i = sum_k alpha[i][k] u_k + beta[i][k] dt L(u_k)
 * (the paper's integrator, Section 7.5); coefficients as published. */
static const double SSP54_A[5][5] = {
    {1.0, 0, 0, 0, 0},
    {0.444370493651235, 0.555629506348765, 0, 0, 0},
    {0.620101851488403, 0, 0.379898148511597, 0, 0},
    {0.178079954393132, 0, 0, 0.821920045606868, 0},
    {0, 0, 0.517231671970585, 0.096059710526147, 0.386708617503269}};
static const double SSP54_B[5][5] = {
    {0.391752226571890, 0, 0, 0, 0},
    {0, 0.368410593050371, 0, 0, 0},
    {0, 0, 0.251891774271694, 0, 0},
    {0, 0, 0, 0.544974750228521, 0},
    {0, 0, 0, 0.063692468666290, 0.226007483236906}};

void ora_ssp54_table(double alpha[25], double beta[25])
{
    for (int i = 0; i < 5; ++i)
        for (int k = 0; k < 5; ++k) {
            alpha[i * 5 + k] = SSP54_A[i][k];
            beta[i * 5 + k] = SSP54_B[i][k];
        }
}

void ora_ssp54(const ora_mesh *m, const ora_phys *ph, double *Q, double dt, int nsteps)
{
    const long n = 5 * m->E * m->np;
    double *u[5], *L[5];
    for (int k = 0; k < 5; ++k) {
        u[k] = malloc(sizeof(double) * n);
        L[k] = malloc(sizeof(double) * n);
        if (!u[k] || !L[k])
            abort();
    }
    for (int st = 0; st < nsteps; ++st) {
        memcpy(u[0], Q, sizeof(double) * n);
        for (int i = 0; i < 5; ++i) {
            /* stage i + 1 from the stages 0..i */
            ora_residual(m, ph, u[i], L[i]);
            double *out = (i < 4) ? u[i + 1] : Q;
            for (long t = 0; t < n; ++t) {
                double s = 0.0;
                for (int k = 0; k <= i; ++k)
                    s += SSP54_A[i][k] * u[k][t] + SSP54_B[i][k] * dt * L[k][t];
                out[t] = s;
            }
        }
    }
    for (int k = 0; k < 5; ++k) {
        free(u[k]);
        free(L[k]);
    }
}

/* Angular-momentum bookkeeping of Section 6: out = (L_x, L_y, L_z, I_x, I_y,
 * I_z), L = integral of rho r x u (the spherical-coordinate integrands of
 * the paper written with x = r sin(theta) cos(phi), y = r sin(theta)
 * sin(phi), z = r cos(theta)), I_x = integral of rho (y^2 + z^2) and so on;
 * quadrature over the solution points with weights w w w |J|, serial order. */
void ora_angular_momentum(const ora_mesh *m, const double *Q, double out[6])
{
    const long E = m->E;
    const int np = m->np, N = m->N;
    for (int k = 0; k < 6; ++k)
        out[k] = 0.0;
    for (long e = 0; e < E; ++e)
        for (int p = 0; p < np; ++p) {
            const int i = p % N, j = (p / N) % N, k = p / (N * N);
            const double wJ = m->w[i] * m->w[j] * m->w[k] * m->jac[e * np + p];
            const double *x = &m->xsol[(e * np + p) * 3];
            const double rho = Q[(0 * E + e) * np + p];
            const double mx = Q[(1 * E + e) * np + p], my = Q[(2 * E + e) * np + p], mz = Q[(3 * E + e) * np + p];
            out[0] += wJ * (x[1] * mz - x[2] * my);
            out[1] += wJ * (x[2] * mx - x[0] * mz);
            out[2] += wJ * (x[0] * my - x[1] * mx);
            out[3] += wJ * rho * (x[1] * x[1] + x[2] * x[2]);
            out[4] += wJ * rho * (x[0] * x[0] + x[2] * x[2]);
            out[5] += wJ * rho * (x[0] * x[0] + x[1] * x[1]);
        }
}

/* Section 6, step 2: remove the rigid rotation dOmega_i = L_i / I_i,
 * u_new = u - dOmega x r at every solution point (the paper's atan2 forms
 * reduce to the components of dOmega x r); density and pressure are kept,
 * so the total energy changes by the change of the kinetic energy.
 * dOmega (may be NULL) receives the applied rates. */
void ora_am_correct(const ora_mesh *m, double *Q, double dOmega[3])
{
    double LI[6], dO[3];
    const long E = m->E;
    const int np = m->np;
    ora_angular_momentum(m, Q, LI);
    for (int c = 0; c < 3; ++c)
        dO[c] = LI[c] / LI[3 + c];
    for (long e = 0; e < E; ++e)
        for (int p = 0; p < np; ++p) {
            const double *x = &m->xsol[(e * np + p) * 3];
            double *q[5];
            for (int v = 0; v < 5; ++v)
                q[v] = &Q[((long)v * E + e) * np + p];
            const double rho = *q[0];
            const double u[3] = {*q[1] / rho, *q[2] / rho, *q[3] / rho};
            const double un[3] = {u[0] - (dO[1] * x[2] - dO[2] * x[1]),
                                  u[1] - (dO[2] * x[0] - dO[0] * x[2]),
                                  u[2] - (dO[0] * x[1] - dO[1] * x[0])};
            const double ke_old = 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            const double ke_new = 0.5 * rho * (un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
            for (int c = 0; c < 3; ++c)
                *q[1 + c] = rho * un[c];
            *q[4] += ke_new - ke_old;
        }
    if (dOmega)
        for (int c = 0; c < 3; ++c)
            dOmega[c] = dO[c];
}

void ora_sums(const ora_mesh *m, const double *Q, double out[5])
{
    int N = m->N;
    for (int v = 0; v < 5; ++v) {
        double s = 0.0;
        for (long e = 0; e < m->E; ++e)
            for (int p = 0; p < m->np; ++p) {
                int i = p % N, j = (p / N) % N, k = p / (N * N);
                s += m->w[i] * m->w[j] * m->w[k] * m->jac[e * m->np + p] * Q[((long)v * m->E + e) * m->np + p];
            }
        out[v] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* polytropic reference state (Section 4.2)                                  */
/* ------------------------------------------------------------------------ */
void ora_polytrope(const ora_mesh *m, double beta, double n_rho, double poly_n, double gamma,
                   double R_gas, const double *noise, double amp, double *Q, double pars[4])
{
    double d = 1.0;
    double chi_o = (beta + 1.0) / (beta * exp(n_rho / poly_n) + 1.0);
    double c = (2.0 * chi_o - beta - 1.0) / (1.0 - beta);
    double alpha = (1.0 + beta) * (1.0 - chi_o) / ((1.0 - beta) * (1.0 - beta));
    double rho_c = 1.0, p_c = 1.0;
    /* hydrostatic balance dp/dr = -rho GM / r^2 of p_c chi^(n+1), rho_c chi^n */
    double GM = (poly_n + 1.0) * alpha * d * p_c / rho_c;
    long n = m->E * m->np;
    for (long g = 0; g < n; ++g) {
        const double *x = &m->xsol[g * 3];
        double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        double chi = c + alpha * d / r;
        double rho = rho_c * pow(chi, poly_n);
        double p = p_c * pow(chi, poly_n + 1.0);
        if (noise)
            rho *= exp(-amp * noise[g]); /* S' = amp c_p noise at fixed p */
        Q[0 * n + g] = rho;
        Q[1 * n + g] = 0.0;
        Q[2 * n + g] = 0.0;
        Q[3 * n + g] = 0.0;
        Q[4 * n + g] = p / (gamma - 1.0);
    }
    (void)R_gas;
    if (pars) {
        pars[0] = chi_o;
        pars[1] = c;
        pars[2] = alpha;
        pars[3] = GM;
    }
}

// Host-side mesh, face table and geometry of the SD library.
//
// Geometry (Section 3: isoparametric 20-node map, transformed fluxes
// |J| J^-1 (F, G, H)):
//   * solution points: x, |J| and |J| grad xi_d = dx/dxi_d1 x dx/dxi_d2 from
//     the exact map derivatives (the chain rule of the viscous gradients is
//     then exact for fields linear in x);
//   * d-flux points: |J| grad xi_d in conservative curl form,
//     (|J| grad xi_d)_n = -(d/dxi_d1 W_d2 - d/dxi_d2 W_d1),
//     W_i = x_l dx_m/dxi_i ((n, m, l) cyclic), with W_i sampled on the lattice
//     of solution points along i and flux points along the two other axes.
//     The tangential derivatives are those of the flux-point polynomials, so
//     the discrete divergence of the metric vanishes (free-stream
//     preservation) and interface area vectors depend only on face data.
//   * interface ends: the side with the larger (element, face) index takes
//     the negated area vector of the other side, so both sides evaluate the
//     same common flux with opposite signs (discrete conservation).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "chorus_internal.hpp"

namespace chorus {

// ---------------------------------------------------------------------------
// 1D operators
// ---------------------------------------------------------------------------
// Legendre P_n on [0,1] and its derivative from the three-term recursion
// P_n = (2n-1)/n (2x-1) P_{n-1} - (n-1)/n P_{n-2}.
static void legendre_pd(int n, double x, double &p, double &dp) {
    double p0 = 1.0, p1 = 0.0, d0 = 0.0, d1 = 0.0;  // P_k, P_{k-1}
    for (int k = 1; k <= n; ++k) {
        double a = (2.0 * k - 1.0) / k, b = (k - 1.0) / k, t = 2.0 * x - 1.0;
        double pk = a * t * p0 - b * p1;
        double dk = a * (2.0 * p0 + t * d0) - b * d1;
        p1 = p0; p0 = pk;
        d1 = d0; d0 = dk;
    }
    p = p0;
    dp = d0;
}

bool build_basis(int N, Basis1D &b) {
    if (N < 2 || N > kMaxOrder) return false;
    b = Basis1D();
    b.N = N;
    for (int s = 0; s < N; ++s) b.xs[s] = 0.5 * (1.0 - std::cos((2.0 * s + 1.0) * M_PI / (2.0 * N)));
    // Legendre-Gauss roots of P_{N-1} by Newton from cosine guesses
    int nr = N - 1;
    b.xf[0] = 0.0;
    b.xf[N] = 1.0;
    std::vector<double> roots;
    for (int k = 0; k < nr; ++k) {
        double x = 0.5 * (1.0 - std::cos(M_PI * (k + 0.75) / (nr + 0.5)));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre_pd(nr, x, p, dp);
            double dx = p / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        roots.push_back(x);
    }
    std::sort(roots.begin(), roots.end());
    for (int k = 0; k < nr; ++k) b.xf[k + 1] = roots[k];
    // barycentric weights
    auto bary = [](const double *X, int n, double *lam) {
        for (int i = 0; i < n; ++i) {
            double v = 1.0;
            for (int j = 0; j < n; ++j)
                if (j != i) v *= (X[i] - X[j]);
            lam[i] = 1.0 / v;
        }
    };
    double ls[kMaxOrder], lf[kMaxOrder + 1];
    bary(b.xs, N, ls);
    bary(b.xf, N + 1, lf);
    // I[m][s] = h_s(xf[m]) = omega_s(x) lam_s / (x - xs[s]); no flux point
    // coincides with a solution point.
    for (int m = 0; m <= N; ++m) {
        double x = b.xf[m], om = 1.0;
        for (int q = 0; q < N; ++q) om *= (x - b.xs[q]);
        for (int s = 0; s < N; ++s) b.I[m][s] = om * ls[s] / (x - b.xs[s]);
    }
    // D[s][m] = l_m'(xs[s]) = l_m(x) * sum_{q != m} 1 / (x - xf[q])
    for (int s = 0; s < N; ++s) {
        double x = b.xs[s], om = 1.0;
        for (int q = 0; q <= N; ++q) om *= (x - b.xf[q]);
        for (int m = 0; m <= N; ++m) {
            double lm = om * lf[m] / (x - b.xf[m]), sum = 0.0;
            for (int q = 0; q <= N; ++q)
                if (q != m) sum += 1.0 / (x - b.xf[q]);
            b.D[s][m] = lm * sum;
        }
    }
    // w_s = int_0^1 h_s: Gauss-Legendre rule on the flux-point roots (exact
    // for degree 2N-3 >= N-1), weights from 1 / ((1-t^2) P'(t)^2) mapped.
    for (int s = 0; s < N; ++s) b.w[s] = 0.0;
    for (int k = 1; k < N; ++k) {
        double x = b.xf[k], p, dp;
        legendre_pd(nr, x, p, dp);
        // derivative wrt t in [-1,1] is dp / 2
        double t = 2.0 * x - 1.0, dpt = 0.5 * dp;
        double wk = 0.5 * 2.0 / ((1.0 - t * t) * dpt * dpt);
        double om = 1.0;
        for (int q = 0; q < N; ++q) om *= (x - b.xs[q]);
        for (int s = 0; s < N; ++s) b.w[s] += wk * om * ls[s] / (x - b.xs[s]);
    }
    return true;
}

// ---------------------------------------------------------------------------
// shell generator (equiangular cubed sphere)
// ---------------------------------------------------------------------------
static const int kLoc[20][3] = {
    {0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {2, 2, 0}, {0, 0, 2}, {2, 0, 2}, {0, 2, 2}, {2, 2, 2},
    {1, 0, 0}, {1, 2, 0}, {1, 0, 2}, {1, 2, 2}, {0, 1, 0}, {2, 1, 0}, {0, 1, 2}, {2, 1, 2},
    {0, 0, 1}, {2, 0, 1}, {0, 2, 1}, {2, 2, 1}};

struct Key4 {
    int64_t v[4];
    bool operator==(const Key4 &o) const { return std::memcmp(v, o.v, sizeof v) == 0; }
};
struct Key4Hash {
    size_t operator()(const Key4 &k) const {
        uint64_t h = 1469598103934665603ull;
        for (int i = 0; i < 4; ++i) {
            h ^= (uint64_t)k.v[i] + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
            h *= 1099511628211ull;
        }
        return (size_t)h;
    }
};

int build_shell(const chorus_shell_desc &d, Mesh &m) {
    const int n = d.panel_n, nr = d.radial_n;
    if (n < 1 || nr < 1 || !(d.r_inner > 0.0) || !(d.r_outer > d.r_inner)) {
        set_error("shell: need panel_n >= 1, radial_n >= 1, 0 < r_inner < r_outer");
        return CHORUS_EINVAL;
    }
    static const int panels[6][4] = {{0, 1, 1, 2}, {0, -1, 1, 2}, {1, 1, 0, 2},
                                     {1, -1, 0, 2}, {2, 1, 0, 1}, {2, -1, 0, 1}};
    const int n2 = 2 * n;
    std::unordered_map<Key4, int64_t, Key4Hash> ids;
    std::vector<Key4> keys;
    const int64_t E = 6LL * n * n * nr;
    m.elem20.assign(E * 20, 0);
    m.face_bc.assign(E * 6, CHORUS_BC_INTERIOR);
    int64_t e = 0;
    for (int pnl = 0; pnl < 6; ++pnl) {
        int axis = panels[pnl][0], sign = panels[pnl][1], ua = panels[pnl][2], va = panels[pnl][3];
        double eu[3] = {0, 0, 0}, ev[3] = {0, 0, 0};
        eu[ua] = 1;
        ev[va] = 1;
        double cr[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2],
                        eu[0] * ev[1] - eu[1] * ev[0]};
        bool flip = cr[axis] * sign < 0;
        for (int k = 0; k < nr; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i, ++e) {
                    for (int c = 0; c < 20; ++c) {
                        int a = 2 * i + kLoc[c][0];
                        if (flip) a = n2 - a;
                        int b = 2 * j + kLoc[c][1];
                        int kk = 2 * k + kLoc[c][2];
                        Key4 key;
                        int64_t cube[3] = {0, 0, 0};
                        cube[axis] = (int64_t)sign * n;
                        cube[ua] = a - n;
                        cube[va] = b - n;
                        key.v[0] = cube[0];
                        key.v[1] = cube[1];
                        key.v[2] = cube[2];
                        key.v[3] = kk;
                        auto it = ids.find(key);
                        int64_t id;
                        if (it == ids.end()) {
                            id = (int64_t)keys.size();
                            ids.emplace(key, id);
                            keys.push_back(key);
                        } else {
                            id = it->second;
                        }
                        m.elem20[e * 20 + c] = id;
                    }
                    if (k == 0) m.face_bc[e * 6 + 4] = CHORUS_BC_INNER;
                    if (k == nr - 1) m.face_bc[e * 6 + 5] = CHORUS_BC_OUTER;
                }
    }
    m.xyz.assign(keys.size() * 3, 0.0);
    for (size_t id = 0; id < keys.size(); ++id) {
        const Key4 &k = keys[id];
        int axis = 0;
        for (int t = 0; t < 3; ++t)
            if (std::llabs(k.v[t]) == n) { axis = t; break; }
        double dir[3];
        for (int t = 0; t < 3; ++t)
            dir[t] = (t == axis) ? (k.v[t] > 0 ? 1.0 : -1.0)
                                 : std::tan(0.25 * M_PI * (double)k.v[t] / n);
        double nrm = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
        double r = d.r_inner + (d.r_outer - d.r_inner) * (double)k.v[3] / (2.0 * nr);
        for (int t = 0; t < 3; ++t) m.xyz[id * 3 + t] = r * (dir[t] / nrm);
    }
    m.match_id.resize(keys.size());
    for (size_t id = 0; id < keys.size(); ++id) m.match_id[id] = (int64_t)id;
    m.E = E;
    m.N = d.order;
    return CHORUS_OK;
}

int build_from_hex20(const chorus_hex20_desc &d, Mesh &m) {
    if (!d.xyz || !d.elem20 || !d.face_bc || d.n_nodes <= 0 || d.n_elems <= 0) {
        set_error("hex20: null array or empty mesh");
        return CHORUS_EINVAL;
    }
    m.N = d.order;
    m.E = d.n_elems;
    m.xyz.assign(d.xyz, d.xyz + d.n_nodes * 3);
    m.elem20.assign(d.elem20, d.elem20 + d.n_elems * 20);
    m.face_bc.assign(d.face_bc, d.face_bc + d.n_elems * 6);
    m.match_id.resize(d.n_nodes);
    for (int64_t i = 0; i < d.n_nodes; ++i) m.match_id[i] = d.match_id ? d.match_id[i] : i;
    for (int64_t i = 0; i < d.n_elems * 20; ++i)
        if (m.elem20[i] < 0 || m.elem20[i] >= d.n_nodes) {
            set_error("hex20: node index out of range");
            return CHORUS_EINVAL;
        }
    for (int64_t i = 0; i < d.n_elems * 6; ++i) {
        int b = m.face_bc[i];
        if (b != CHORUS_BC_INTERIOR && b != CHORUS_BC_INNER && b != CHORUS_BC_OUTER &&
            b != CHORUS_BC_STATE) {
            set_error("hex20: unknown face tag");
            return CHORUS_EINVAL;
        }
    }
    return CHORUS_OK;
}

// ---------------------------------------------------------------------------
// faces
// ---------------------------------------------------------------------------
// local corner of face f at face-local corner (c1, c2); c1, c2 run along the
// two tangential axes in increasing axis order
static int corner_of_face(int f, int c1, int c2) {
    int d = f >> 1, side = f & 1, ijk[3];
    ijk[d] = side;
    int t = 0;
    for (int ax = 0; ax < 3; ++ax)
        if (ax != d) ijk[ax] = (t++ == 0) ? c1 : c2;
    return ijk[0] + 2 * ijk[1] + 4 * ijk[2];
}

static int build_faces(Mesh &m) {
    const int64_t E = m.E;
    m.links.assign(E * 6, FaceLink());
    std::unordered_map<Key4, int64_t, Key4Hash> open;
    open.reserve((size_t)(E * 3));
    m.n_faces = 0;
    m.n_wall_faces = 0;
    auto corner_id = [&](int64_t e, int f, int c1, int c2) {
        return m.match_id[m.elem20[e * 20 + corner_of_face(f, c1, c2)]];
    };
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            FaceLink &L = m.links[e * 6 + f];
            L.bc = m.face_bc[e * 6 + f];
            if (L.bc != CHORUS_BC_INTERIOR) {
                ++m.n_faces;
                if (L.bc == CHORUS_BC_INNER || L.bc == CHORUS_BC_OUTER) ++m.n_wall_faces;
                continue;
            }
            Key4 k;
            k.v[0] = corner_id(e, f, 0, 0);
            k.v[1] = corner_id(e, f, 1, 0);
            k.v[2] = corner_id(e, f, 0, 1);
            k.v[3] = corner_id(e, f, 1, 1);
            std::sort(k.v, k.v + 4);
            auto it = open.find(k);
            if (it == open.end()) {
                open.emplace(k, e * 6 + f);
                continue;
            }
            int64_t other = it->second;
            open.erase(it);
            int64_t e2 = other / 6;
            int f2 = (int)(other % 6);
            // orientation of this face seen from each side
            for (int pass = 0; pass < 2; ++pass) {
                int64_t ea = pass ? e2 : e, eb = pass ? e : e2;
                int fa = pass ? f2 : f, fb = pass ? f : f2;
                int pos[2][2][2];  // our corner (c1,c2) -> neighbour (u1,u2)
                for (int c2 = 0; c2 < 2; ++c2)
                    for (int c1 = 0; c1 < 2; ++c1) {
                        int64_t id = corner_id(ea, fa, c1, c2);
                        int hits = 0;
                        for (int u2 = 0; u2 < 2; ++u2)
                            for (int u1 = 0; u1 < 2; ++u1)
                                if (corner_id(eb, fb, u1, u2) == id) {
                                    pos[c1][c2][0] = u1;
                                    pos[c1][c2][1] = u2;
                                    ++hits;
                                }
                        if (hits != 1) {
                            set_error("degenerate face (repeated corner ids) at element " +
                                      std::to_string(ea));
                            return CHORUS_EMESH;
                        }
                    }
                int flip1 = pos[0][0][0], flip2 = pos[0][0][1];
                int swap = (pos[1][0][1] != pos[0][0][1]) ? 1 : 0;
                // check all four corners against the dihedral map
                for (int c2 = 0; c2 < 2; ++c2)
                    for (int c1 = 0; c1 < 2; ++c1) {
                        int u1 = swap ? c2 : c1, u2 = swap ? c1 : c2;
                        if (flip1) u1 = 1 - u1;
                        if (flip2) u2 = 1 - u2;
                        if (u1 != pos[c1][c2][0] || u2 != pos[c1][c2][1]) {
                            set_error("non-conforming face at element " + std::to_string(ea));
                            return CHORUS_EMESH;
                        }
                    }
                FaceLink &La = m.links[ea * 6 + fa];
                La.nbr_elem = (int32_t)eb;
                La.nbr_face = fb;
                La.orient = swap * 4 + flip1 * 2 + flip2;
            }
            ++m.n_faces;
        }
    if (!open.empty()) {
        int64_t code = open.begin()->second;
        set_error("unmatched interior face: element " + std::to_string(code / 6) + " face " +
                  std::to_string(code % 6));
        return CHORUS_EMESH;
    }
    if (E > INT32_MAX) {
        set_error("too many elements for 32-bit neighbour indices");
        return CHORUS_EINVAL;
    }
    return CHORUS_OK;
}

// neighbour face-point index of our face point (t1, t2) under orientation o
static inline int map_face_point(int o, int N, int t1, int t2) {
    int u1 = (o & 4) ? t2 : t1, u2 = (o & 4) ? t1 : t2;
    if (o & 2) u1 = N - 1 - u1;
    if (o & 1) u2 = N - 1 - u2;
    return u1 + N * u2;
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
// forward-mode dual number with three partial derivatives
struct Dual {
    double v, d[3];
};
static inline Dual dconst(double c) { return Dual{c, {0, 0, 0}}; }
static inline Dual operator+(Dual a, Dual b) {
    return Dual{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]}};
}
static inline Dual operator-(Dual a, Dual b) {
    return Dual{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]}};
}
static inline Dual operator*(Dual a, Dual b) {
    return Dual{a.v * b.v, {a.d[0] * b.v + a.v * b.d[0], a.d[1] * b.v + a.v * b.d[1],
                            a.d[2] * b.v + a.v * b.d[2]}};
}
static inline Dual operator*(double c, Dual a) { return Dual{c * a.v, {c * a.d[0], c * a.d[1], c * a.d[2]}}; }

// the 20 serendipity shape functions at reference point r (derivatives wrt
// xi, eta, zeta on [0,1]^3)
static void shape20(const double r[3], Dual out[20]) {
    Dual a[3];
    for (int t = 0; t < 3; ++t) {
        a[t] = Dual{2.0 * r[t] - 1.0, {0, 0, 0}};
        a[t].d[t] = 2.0;
    }
    for (int n = 0; n < 20; ++n) {
        int p[3] = {kLoc[n][0] - 1, kLoc[n][1] - 1, kLoc[n][2] - 1};
        int zero = -1;
        for (int t = 0; t < 3; ++t)
            if (p[t] == 0) zero = t;
        if (zero < 0) {
            Dual prod = dconst(0.125), sum = dconst(-2.0);
            for (int t = 0; t < 3; ++t) {
                prod = prod * (dconst(1.0) + (double)p[t] * a[t]);
                sum = sum + (double)p[t] * a[t];
            }
            out[n] = prod * sum;
        } else {
            Dual v = 0.25 * (dconst(1.0) - a[zero] * a[zero]);
            for (int t = 0; t < 3; ++t)
                if (t != zero) v = v * (dconst(1.0) + (double)p[t] * a[t]);
            out[n] = v;
        }
    }
}

struct Table {
    std::vector<double> val;  // [pt][20]
    std::vector<double> der;  // [pt][20][3]
};

static void tabulate(const std::vector<std::array<double, 3>> &pts, Table &t) {
    t.val.resize(pts.size() * 20);
    t.der.resize(pts.size() * 60);
    Dual s[20];
    for (size_t q = 0; q < pts.size(); ++q) {
        shape20(pts[q].data(), s);
        for (int n = 0; n < 20; ++n) {
            t.val[q * 20 + n] = s[n].v;
            for (int i = 0; i < 3; ++i) t.der[(q * 20 + n) * 3 + i] = s[n].d[i];
        }
    }
}

static int build_geometry(Mesh &m) {
    const int N = m.N, NP = N * N * N, NFL = (N + 1) * N * N, L = N + 1;
    const Basis1D &b = m.basis;
    const int64_t E = m.E;
    // reference points: solution lattice, then for each axis i the lattice
    // with solution points along i and flux points along the others
    std::vector<std::array<double, 3>> sol_pts(NP);
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) sol_pts[i + N * (j + N * k)] = {b.xs[i], b.xs[j], b.xs[k]};
    const int NW = L * L * L;  // lattice stored in an (N+1)^3 box
    std::vector<std::array<double, 3>> w_pts(3 * NW, {0.5, 0.5, 0.5});
    for (int i = 0; i < 3; ++i)
        for (int a2 = 0; a2 < L; ++a2)
            for (int a1 = 0; a1 < L; ++a1)
                for (int a0 = 0; a0 < L; ++a0) {
                    int idx[3] = {a0, a1, a2};
                    if (idx[i] >= N) continue;
                    std::array<double, 3> r;
                    for (int t = 0; t < 3; ++t) r[t] = (t == i) ? b.xs[idx[t]] : b.xf[idx[t]];
                    w_pts[i * NW + a0 + L * (a1 + L * a2)] = r;
                }
    // d-flux points: flux coordinate along d, solution coordinates along the
    // other two axes (index a + (N+1)(t1 + N t2))
    std::vector<std::array<double, 3>> f_pts(3 * NFL);
    for (int d = 0; d < 3; ++d)
        for (int fl = 0; fl < NFL; ++fl) {
            int a = fl % L, t1 = (fl / L) % N, t2 = fl / (L * N);
            std::array<double, 3> r;
            int t = 0;
            for (int ax = 0; ax < 3; ++ax) r[ax] = (ax == d) ? b.xf[a] : b.xs[(t++ == 0) ? t1 : t2];
            f_pts[d * NFL + fl] = r;
        }
    Table ts, tw, tf;
    tabulate(sol_pts, ts);
    tabulate(w_pts, tw);
    tabulate(f_pts, tf);
    m.rflux.assign(E * 3 * NFL, 0.0);
    m.xsol.assign(E * NP * 3, 0.0);
    m.jac.assign(E * NP, 0.0);
    m.met.assign(E * NP * 9, 0.0);
    m.metf.assign(E * 3 * NFL * 3, 0.0);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t e = 0; e < E; ++e) {
        double X[20][3];
        for (int n = 0; n < 20; ++n)
            for (int c = 0; c < 3; ++c) X[n][c] = m.xyz[m.elem20[e * 20 + n] * 3 + c];
        for (int p = 0; p < NP; ++p) {
            double x[3] = {0, 0, 0}, J[3][3] = {{0}};  // J[c][i] = dx_c / dxi_i
            for (int n = 0; n < 20; ++n) {
                double v = ts.val[p * 20 + n];
                for (int c = 0; c < 3; ++c) {
                    x[c] += v * X[n][c];
                    for (int i = 0; i < 3; ++i) J[c][i] += ts.der[(p * 20 + n) * 3 + i] * X[n][c];
                }
            }
            double det = J[0][0] * (J[1][1] * J[2][2] - J[2][1] * J[1][2]) -
                         J[1][0] * (J[0][1] * J[2][2] - J[2][1] * J[0][2]) +
                         J[2][0] * (J[0][1] * J[1][2] - J[1][1] * J[0][2]);
            if (!(det > 0.0)) bad = 1;
            m.jac[e * NP + p] = det;
            for (int c = 0; c < 3; ++c) m.xsol[(e * NP + p) * 3 + c] = x[c];
            for (int d = 0; d < 3; ++d) {
                int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
                double *o = &m.met[((e * NP + p) * 3 + d) * 3];
                // column d1 cross column d2
                o[0] = J[1][d1] * J[2][d2] - J[2][d1] * J[1][d2];
                o[1] = J[2][d1] * J[0][d2] - J[0][d1] * J[2][d2];
                o[2] = J[0][d1] * J[1][d2] - J[1][d1] * J[0][d2];
            }
        }
        for (int q = 0; q < 3 * NFL; ++q) {
            double x[3] = {0, 0, 0};
            for (int n = 0; n < 20; ++n)
                for (int c = 0; c < 3; ++c) x[c] += tf.val[q * 20 + n] * X[n][c];
            m.rflux[e * 3 * NFL + q] = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        }
        // W[n][i] on lattice i
        std::vector<double> W(9 * NW, 0.0);
        for (int i = 0; i < 3; ++i)
            for (int q = 0; q < NW; ++q) {
                int a0 = q % L, a1 = (q / L) % L, a2 = q / (L * L);
                int idx[3] = {a0, a1, a2};
                if (idx[i] >= N) continue;
                const int pt = i * NW + q;
                double x[3] = {0, 0, 0}, dxi[3] = {0, 0, 0};
                for (int n = 0; n < 20; ++n) {
                    double v = tw.val[pt * 20 + n], dv = tw.der[(pt * 20 + n) * 3 + i];
                    for (int c = 0; c < 3; ++c) {
                        x[c] += v * X[n][c];
                        dxi[c] += dv * X[n][c];
                    }
                }
                for (int nn = 0; nn < 3; ++nn) {
                    int mm = (nn + 1) % 3, l = (nn + 2) % 3;
                    W[(nn * 3 + i) * NW + q] = x[l] * dxi[mm];
                }
            }
        for (int d = 0; d < 3; ++d) {
            int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
            for (int fl = 0; fl < NFL; ++fl) {
                int a = fl % L, t1 = (fl / L) % N, t2 = fl / (L * N);
                int idx[3];
                idx[d] = a;
                int t = 0;
                for (int ax = 0; ax < 3; ++ax)
                    if (ax != d) idx[ax] = (t++ == 0) ? t1 : t2;
                for (int nn = 0; nn < 3; ++nn) {
                    double s1 = 0.0, s2 = 0.0;
                    for (int q = 0; q <= N; ++q) {
                        int j1[3] = {idx[0], idx[1], idx[2]}, j2[3] = {idx[0], idx[1], idx[2]};
                        j1[d1] = q;
                        j2[d2] = q;
                        s1 += b.D[idx[d1]][q] * W[(nn * 3 + d2) * NW + j1[0] + L * (j1[1] + L * j1[2])];
                        s2 += b.D[idx[d2]][q] * W[(nn * 3 + d1) * NW + j2[0] + L * (j2[1] + L * j2[2])];
                    }
                    m.metf[((e * 3 + d) * NFL + fl) * 3 + nn] = s2 - s1;
                }
            }
        }
    }
    if (bad) {
        set_error("non-positive Jacobian at a solution point");
        return CHORUS_EMESH;
    }
    m.rflux_min = m.rflux_max = m.rflux.empty() ? 0.0 : m.rflux[0];
    for (double r : m.rflux) {
        m.rflux_min = std::min(m.rflux_min, r);
        m.rflux_max = std::max(m.rflux_max, r);
    }
    // antisymmetric interface area vectors
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            const FaceLink &Lk = m.links[e * 6 + f];
            if (Lk.nbr_elem < 0) continue;
            int64_t e2 = Lk.nbr_elem;
            int f2 = Lk.nbr_face;
            if (e * 6 + f > e2 * 6 + f2) continue;  // this side owns the face
            int d = f >> 1, d2 = f2 >> 1;
            double sg = (f & 1) ? 1.0 : -1.0, sg2 = (f2 & 1) ? 1.0 : -1.0;
            int a = (f & 1) ? N : 0, a2 = (f2 & 1) ? N : 0;
            for (int t2 = 0; t2 < N; ++t2)
                for (int t1 = 0; t1 < N; ++t1) {
                    int pn = map_face_point(Lk.orient, N, t1, t2);
                    int fl = a + L * (t1 + N * t2), fl2 = a2 + L * (pn % N + N * (pn / N));
                    for (int c = 0; c < 3; ++c) {
                        double Sout = sg * m.metf[((e * 3 + d) * NFL + fl) * 3 + c];
                        m.metf[((e2 * 3 + d2) * NFL + fl2) * 3 + c] = sg2 * (-Sout);
                    }
                }
        }
    return CHORUS_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static void build_image(Mesh &m) {
    const int N = m.N, NP = N * N * N, NFL = (N + 1) * N * N;
    const int64_t E = m.E;
    DeviceLayout &L = m.layout;
    size_t off = 0;
    L.solgeo = off;    off = align256(off + sizeof(double) * E * 13 * NP);
    L.fluxgeo = off;   off = align256(off + sizeof(double) * E * 9 * NFL);
    L.link = off;      off = align256(off + sizeof(int32_t) * E * 6);
    L.info = off;      off = align256(off + sizeof(int32_t) * E * 6);
    L.solw = off;      off = align256(off + sizeof(double) * E * NP);
    L.solgeo32 = off;  off = align256(off + sizeof(float) * E * 13 * NP);
    L.fluxgeo32 = off; off = align256(off + sizeof(float) * E * 9 * NFL);
    L.xsol = off;      off = align256(off + sizeof(double) * E * 3 * NP);
    L.rflux = off;     off = align256(off + sizeof(double) * E * 3 * NFL);
    L.rflux32 = off;   off = align256(off + sizeof(float) * E * 3 * NFL);
    L.total = off;
    m.image.assign(L.total, 0);
    double *sg = (double *)(m.image.data() + L.solgeo);
    double *fg = (double *)(m.image.data() + L.fluxgeo);
    int32_t *lk = (int32_t *)(m.image.data() + L.link);
    int32_t *inf = (int32_t *)(m.image.data() + L.info);
    double *sw = (double *)(m.image.data() + L.solw);
    float *sg32 = (float *)(m.image.data() + L.solgeo32);
    float *fg32 = (float *)(m.image.data() + L.fluxgeo32);
    double *xs = (double *)(m.image.data() + L.xsol);
    const Basis1D &b = m.basis;
    for (int64_t e = 0; e < E; ++e) {
        for (int p = 0; p < NP; ++p) {
            double J = m.jac[e * NP + p];
            for (int d = 0; d < 3; ++d)
                for (int c = 0; c < 3; ++c)
                    sg[(e * 13 + d * 3 + c) * NP + p] = m.met[((e * NP + p) * 3 + d) * 3 + c] / J;
            sg[(e * 13 + 9) * NP + p] = 1.0 / J;
            const double *x = &m.xsol[(e * NP + p) * 3];
            double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            for (int c = 0; c < 3; ++c) sg[(e * 13 + 10 + c) * NP + p] = x[c] / (r * r * r);
            for (int c = 0; c < 3; ++c) xs[(e * 3 + c) * NP + p] = x[c];
            int i = p % N, j = (p / N) % N, k = p / (N * N);
            sw[e * NP + p] = b.w[i] * b.w[j] * b.w[k] * J;
        }
        for (int d = 0; d < 3; ++d)
            for (int c = 0; c < 3; ++c)
                for (int fl = 0; fl < NFL; ++fl)
                    fg[((e * 3 + d) * 3 + c) * NFL + fl] = m.metf[((e * 3 + d) * NFL + fl) * 3 + c];
        for (int f = 0; f < 6; ++f) {
            const FaceLink &Lk = m.links[e * 6 + f];
            lk[e * 6 + f] = Lk.nbr_elem;
            int nf = Lk.nbr_face < 0 ? 0 : Lk.nbr_face, o = Lk.orient < 0 ? 0 : Lk.orient;
            inf[e * 6 + f] = nf | (o << 3) | ((Lk.bc + 1) << 6);
        }
    }
    for (int64_t t = 0; t < E * 13 * NP; ++t) sg32[t] = (float)sg[t];
    for (int64_t t = 0; t < E * 9 * NFL; ++t) fg32[t] = (float)fg[t];
    double *rf = (double *)(m.image.data() + L.rflux);
    float *rf32 = (float *)(m.image.data() + L.rflux32);
    for (int64_t t = 0; t < E * 3 * NFL; ++t) {
        rf[t] = m.rflux[t];
        rf32[t] = (float)m.rflux[t];
    }
}

int finish_mesh(Mesh &m) {
    if (!build_basis(m.N, m.basis)) {
        set_error("order must be in [2, 6]");
        return CHORUS_EINVAL;
    }
    int rc = build_faces(m);
    if (rc) return rc;
    rc = build_geometry(m);
    if (rc) return rc;
    build_image(m);
    return CHORUS_OK;
}

}  // namespace chorus

// Host side of build_geometry: validation of the NURBS patches (Sec. 3.2),
// per-element rational Bezier extraction, the spline spaces of Sec. 3.3 and the
// gluing of S^0.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <numeric>
#include <sched.h>
#include <unordered_map>

#include "common.h"

namespace igb {

namespace {

thread_local char g_err[1024] = "";

// Blossom of a degree-p B-spline segment: control values d[0..p] (dimension
// dim) are the coefficients of b_{s-p..s} on knot span s, args[0..p-1] the
// blossom arguments.  With all arguments equal this is de Boor's algorithm.
void blossom(const double* knots, int s, int p, const double* args, const double* d, int dim,
             double* out) {
    double w[(PGMAX + 1) * 4];
    for (int i = 0; i < (p + 1) * dim; ++i) w[i] = d[i];
    for (int r = 1; r <= p; ++r) {
        for (int j = p; j >= r; --j) {
            int kj = s - p + j;  // knot index of the control value
            double den = knots[kj + p + 1 - r] - knots[kj];
            double a = den > 0 ? (args[r - 1] - knots[kj]) / den : 0.0;
            for (int c = 0; c < dim; ++c)
                w[j * dim + c] = (1.0 - a) * w[(j - 1) * dim + c] + a * w[j * dim + c];
        }
    }
    for (int c = 0; c < dim; ++c) out[c] = w[p * dim + c];
}

// Bezier coefficients of the segment of span s restricted to [a, b]: the
// blossom values f(a^{p-i}, b^i), i = 0..p.
void bezier_on_interval(const double* knots, int s, int p, double a, double b, const double* d,
                        int dim, double* out /*[(p+1)*dim]*/) {
    double args[PGMAX];
    for (int i = 0; i <= p; ++i) {
        for (int r = 0; r < p; ++r) args[r] = r < p - i ? a : b;
        blossom(knots, s, p, args, d, dim, out + i * dim);
    }
}

int find_span(const std::vector<double>& kn, int p, int ncp, double a, double b) {
    for (int s = p; s < ncp; ++s)
        if (kn[s] <= a && kn[s + 1] >= b && kn[s] < kn[s + 1]) return s;
    return -1;
}

struct UnionFind {
    std::vector<int> par;
    explicit UnionFind(size_t n) : par(n) { std::iota(par.begin(), par.end(), 0); }
    int find(int i) {
        while (par[i] != i) i = par[i] = par[par[i]];
        return i;
    }
    void unite(int a, int b) {
        a = find(a);
        b = find(b);
        if (a != b) par[std::max(a, b)] = std::min(a, b);
    }
};

// Points closer than tol get the same label (spatial hashing on cells of size
// tol*1e3, neighbours searched in the 27 adjacent cells).
std::vector<int> match_points(const std::vector<double>& pts, double tol) {
    size_t n = pts.size() / 3;
    UnionFind uf(n);
    double cell = tol * 1e3;
    struct Key {
        int64_t a, b, c;
        bool operator==(const Key& o) const { return a == o.a && b == o.b && c == o.c; }
    };
    struct H {
        size_t operator()(const Key& k) const {
            return std::hash<int64_t>()(k.a * 73856093LL ^ k.b * 19349663LL ^ k.c * 83492791LL);
        }
    };
    std::unordered_map<Key, std::vector<int>, H> grid;
    grid.reserve(n * 2);
    for (size_t i = 0; i < n; ++i) {
        Key k{(int64_t)std::floor(pts[3 * i] / cell), (int64_t)std::floor(pts[3 * i + 1] / cell),
              (int64_t)std::floor(pts[3 * i + 2] / cell)};
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    auto it = grid.find(Key{k.a + dx, k.b + dy, k.c + dz});
                    if (it == grid.end()) continue;
                    for (int j : it->second) {
                        double d0 = pts[3 * i] - pts[3 * j], d1 = pts[3 * i + 1] - pts[3 * j + 1],
                               d2 = pts[3 * i + 2] - pts[3 * j + 2];
                        if (d0 * d0 + d1 * d1 + d2 * d2 <= tol * tol) uf.unite((int)i, j);
                    }
                }
        grid[k].push_back((int)i);
    }
    std::vector<int> lab(n);
    for (size_t i = 0; i < n; ++i) lab[i] = uf.find((int)i);
    return lab;
}

void bernstein_host(int p, double s, double* b, double* db) {
    // explicit Bernstein polynomials of degree p <= 3 on [0,1] and derivatives
    double t = 1.0 - s;
    switch (p) {
        case 0: b[0] = 1; db[0] = 0; break;
        case 1: b[0] = t; b[1] = s; db[0] = -1; db[1] = 1; break;
        case 2:
            b[0] = t * t; b[1] = 2 * s * t; b[2] = s * s;
            db[0] = -2 * t; db[1] = 2 * (t - s); db[2] = 2 * s;
            break;
        default:
            b[0] = t * t * t; b[1] = 3 * s * t * t; b[2] = 3 * s * s * t; b[3] = s * s * s;
            db[0] = -3 * t * t; db[1] = 3 * t * t - 6 * s * t; db[2] = 6 * s * t - 3 * s * s;
            db[3] = 3 * s * s;
    }
}

}  // namespace

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

const char* last_error() { return g_err; }

int host_threads() {
    cpu_set_t set;
    CPU_ZERO(&set);
    const int n = sched_getaffinity(0, sizeof(set), &set) == 0 ? CPU_COUNT(&set) : 1;
    return std::max(1, std::min(n, 16));
}

void cheb_nodes(int q, double* t) {
    for (int k = 0; k <= q; ++k) t[k] = 0.5 * (1.0 - std::cos((2 * k + 1) * M_PI / (2 * q + 2)));
}

// Evaluates F and its derivatives w.r.t. the element-local coordinates at
// (s, t) from the element's homogeneous Bezier net (host).
void eval_element_host(const igb_geom_s* g, int64_t e, double s, double t, double* F, double* Fs,
                       double* Ft) {
    int pu = g->pg[2 * e], pv = g->pg[2 * e + 1];
    double bu[4], dbu[4], bv[4], dbv[4];
    bernstein_host(pu, s, bu, dbu);
    bernstein_host(pv, t, bv, dbv);
    double P[4] = {0, 0, 0, 0}, Ps[4] = {0, 0, 0, 0}, Pt[4] = {0, 0, 0, 0};
    const double* H = &g->bez[e * NBZ * 4];
    for (int j = 0; j <= pv; ++j)
        for (int i = 0; i <= pu; ++i)
            for (int c = 0; c < 4; ++c) {
                double h = H[(j * (PGMAX + 1) + i) * 4 + c];
                P[c] += bv[j] * bu[i] * h;
                Ps[c] += bv[j] * dbu[i] * h;
                Pt[c] += dbv[j] * bu[i] * h;
            }
    for (int c = 0; c < 3; ++c) {
        F[c] = P[c] / P[3];
        if (Fs) Fs[c] = (Ps[c] - F[c] * Ps[3]) / P[3];
        if (Ft) Ft[c] = (Pt[c] - F[c] * Pt[3]) / P[3];
    }
}

igb_status geometry_build(igb_ctx ctx, const igb_patch* patches, int npatch, int m, int p,
                          igb_geom g) {
    if (npatch <= 0 || m < 0 || m > 12 || p < 0 || p > PMAX) {
        set_error("build_geometry: need npatch > 0, 0 <= m <= 12, 0 <= p <= %d", PMAX);
        return IGB_ERR_ARG;
    }
    g->ctx = ctx;
    g->npatch = npatch;
    g->m = m;
    g->p = p;
    g->nel1 = 1 << m;
    g->k = g->nel1 + p;
    const int nel1 = g->nel1;
    g->nelem = int64_t(npatch) * nel1 * nel1;
    g->n2 = int64_t(npatch) * g->k * g->k;
    const int64_t E = g->nelem;
    g->bez.assign(E * NBZ * 4, 0.0);
    g->pg.assign(E * 2, 0);
    g->lo.assign(E * 3, 0.0);
    g->espan.assign(E * 2, 0);
    g->hi.assign(E * 3, 0.0);
    g->corner.assign(E * 12, 0.0);
    const double h = 1.0 / nel1;

    for (int j = 0; j < npatch; ++j) {
        const igb_patch& P = patches[j];
        if (P.deg_u < 0 || P.deg_u > PGMAX || P.deg_v < 0 || P.deg_v > PGMAX || P.ncp_u <= P.deg_u ||
            P.ncp_v <= P.deg_v || !P.knots_u || !P.knots_v || !P.cpw) {
            set_error("build_geometry: patch %d has degree > %d or too few control points", j, PGMAX);
            return IGB_ERR_ARG;
        }
        std::vector<double> ku(P.knots_u, P.knots_u + P.ncp_u + P.deg_u + 1);
        std::vector<double> kv(P.knots_v, P.knots_v + P.ncp_v + P.deg_v + 1);
        for (auto* kn : {&ku, &kv}) {
            int deg = kn == &ku ? P.deg_u : P.deg_v;
            for (size_t i = 1; i < kn->size(); ++i)
                if ((*kn)[i] < (*kn)[i - 1]) {
                    set_error("build_geometry: patch %d knots not non-decreasing", j);
                    return IGB_ERR_GEOMETRY;
                }
            for (int i = 0; i <= deg; ++i)
                if ((*kn)[i] != 0.0 || (*kn)[kn->size() - 1 - i] != 1.0) {
                    set_error("build_geometry: patch %d knot vector is not open on [0,1]", j);
                    return IGB_ERR_GEOMETRY;
                }
            for (size_t i = deg + 1; i + deg + 1 < kn->size(); ++i) {
                double x = (*kn)[i] * nel1;
                if (std::fabs(x - std::round(x)) > 1e-12) {
                    set_error("build_geometry: patch %d knot %g is not a mesh knot j/2^m", j, (*kn)[i]);
                    return IGB_ERR_GEOMETRY;
                }
            }
        }
        const int nu = P.ncp_u, nv = P.ncp_v;
        std::vector<double> hom(size_t(nu) * nv * 4);
        for (int b = 0; b < nv; ++b)
            for (int a = 0; a < nu; ++a) {
                const double* c = P.cpw + (size_t(b) * nu + a) * 4;
                if (!(c[3] > 0)) {
                    set_error("build_geometry: patch %d has a weight <= 0", j);
                    return IGB_ERR_GEOMETRY;
                }
                for (int x = 0; x < 3; ++x) hom[(size_t(b) * nu + a) * 4 + x] = c[x] * c[3];
                hom[(size_t(b) * nu + a) * 4 + 3] = c[3];
            }
        for (int ey = 0; ey < nel1; ++ey)
            for (int ex = 0; ex < nel1; ++ex) {
                const int64_t e = (int64_t(j) * nel1 + ey) * nel1 + ex;
                double u0 = ex * h, u1 = (ex + 1) * h, v0 = ey * h, v1 = (ey + 1) * h;
                int su = find_span(ku, P.deg_u, nu, u0, u1), sv = find_span(kv, P.deg_v, nv, v0, v1);
                if (su < 0 || sv < 0) {
                    set_error("build_geometry: element not inside one knot span (patch %d)", j);
                    return IGB_ERR_GEOMETRY;
                }
                g->espan[2 * e] = su;
                g->espan[2 * e + 1] = sv;
                const int pu = P.deg_u, pv = P.deg_v;
                // u-direction first: rows b = sv-pv..sv give Bezier nets in u
                double rowbez[PGMAX + 1][(PGMAX + 1) * 4];
                for (int r = 0; r <= pv; ++r) {
                    int b = sv - pv + r;
                    double d[(PGMAX + 1) * 4];
                    for (int i = 0; i <= pu; ++i)
                        for (int c = 0; c < 4; ++c) d[i * 4 + c] = hom[(size_t(b) * nu + su - pu + i) * 4 + c];
                    bezier_on_interval(ku.data(), su, pu, u0, u1, d, 4, rowbez[r]);
                }
                // then v for every u-Bezier index
                for (int i = 0; i <= pu; ++i) {
                    double d[(PGMAX + 1) * 4], out[(PGMAX + 1) * 4];
                    for (int r = 0; r <= pv; ++r)
                        for (int c = 0; c < 4; ++c) d[r * 4 + c] = rowbez[r][i * 4 + c];
                    bezier_on_interval(kv.data(), sv, pv, v0, v1, d, 4, out);
                    for (int r = 0; r <= pv; ++r)
                        for (int c = 0; c < 4; ++c)
                            g->bez[(e * NBZ + r * (PGMAX + 1) + i) * 4 + c] = out[r * 4 + c];
                }
                g->pg[2 * e] = pu;
                g->pg[2 * e + 1] = pv;
                double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
                for (int r = 0; r <= pv; ++r)
                    for (int i = 0; i <= pu; ++i) {
                        const double* H = &g->bez[(e * NBZ + r * (PGMAX + 1) + i) * 4];
                        if (!(H[3] > 0)) {
                            set_error("build_geometry: non-positive Bezier weight");
                            return IGB_ERR_GEOMETRY;
                        }
                        for (int c = 0; c < 3; ++c) {
                            lo[c] = std::min(lo[c], H[c] / H[3]);
                            hi[c] = std::max(hi[c], H[c] / H[3]);
                        }
                    }
                for (int c = 0; c < 3; ++c) {
                    g->lo[3 * e + c] = lo[c];
                    g->hi[3 * e + c] = hi[c];
                }
                const int cu[4] = {0, pu, 0, pu}, cv[4] = {0, 0, pv, pv};
                for (int cc = 0; cc < 4; ++cc) {
                    const double* H = &g->bez[(e * NBZ + cv[cc] * (PGMAX + 1) + cu[cc]) * 4];
                    for (int c = 0; c < 3; ++c) g->corner[e * 12 + cc * 3 + c] = H[c] / H[3];
                }
            }
    }

    // global vertex ids by matching corner points
    double diam = 0;
    for (int c = 0; c < 3; ++c) {
        double a = 1e300, b = -1e300;
        for (int64_t e = 0; e < E; ++e) {
            a = std::min(a, g->lo[3 * e + c]);
            b = std::max(b, g->hi[3 * e + c]);
        }
        diam = std::max(diam, b - a);
    }
    const double tol = 1e-9 * diam;
    g->vert = match_points(g->corner, tol);

    // closed, consistently oriented surface: every directed element edge has its
    // reverse in exactly one other element (local order (0,0)->(1,0)->(1,1)->(0,1))
    {
        std::unordered_map<int64_t, int> cnt;
        cnt.reserve(E * 8);
        auto key = [](int64_t a, int64_t b) { return a * 4294967296LL + b; };
        const int ring[4] = {0, 1, 3, 2};
        for (int64_t e = 0; e < E; ++e)
            for (int k = 0; k < 4; ++k) {
                int a = g->vert[4 * e + ring[k]], b = g->vert[4 * e + ring[(k + 1) % 4]];
                cnt[key(a, b)]++;
            }
        for (auto& kv : cnt) {
            int64_t a = kv.first >> 32, b = kv.first & 0xffffffffLL;
            auto it = cnt.find(key(b, a));
            if (kv.second != 1 || it == cnt.end() || it->second != 1) {
                set_error("build_geometry: surface is not closed or patches are not consistently "
                          "oriented / conforming");
                return IGB_ERR_GEOMETRY;
            }
        }
    }
    // outward orientation: enclosed volume (1/3) int F . n~ > 0
    {
        const double gx[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
        double vol = 0;
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    double F[3], Fs[3], Ft[3];
                    eval_element_host(g, e, gx[a], gx[b], F, Fs, Ft);
                    double n[3] = {Fs[1] * Ft[2] - Fs[2] * Ft[1], Fs[2] * Ft[0] - Fs[0] * Ft[2],
                                   Fs[0] * Ft[1] - Fs[1] * Ft[0]};
                    vol += 0.25 * (F[0] * n[0] + F[1] * n[1] + F[2] * n[2]) / 3.0;
                }
        if (!(vol > 0)) {
            set_error("build_geometry: normals d_uF x d_vF point into the enclosed volume");
            return IGB_ERR_GEOMETRY;
        }
    }

    // 1-D extraction of the B-splines of Xi_{p,m} on each element
    {
        std::vector<double> kn(size_t(g->k) + p + 1);
        for (int i = 0; i <= p; ++i) {
            kn[i] = 0.0;
            kn[kn.size() - 1 - i] = 1.0;
        }
        for (int i = 1; i < nel1; ++i) kn[p + i] = double(i) / nel1;
        g->C1.assign(size_t(nel1) * (p + 1) * (p + 1), 0.0);
        for (int ex = 0; ex < nel1; ++ex) {
            int s = ex + p;
            for (int a = 0; a <= p; ++a) {
                double d[PMAX + 1] = {0, 0, 0, 0};
                d[a] = 1.0;
                double out[PMAX + 1];
                bezier_on_interval(kn.data(), s, p, ex * h, (ex + 1) * h, d, 1, out);
                for (int kk = 0; kk <= p; ++kk) g->C1[(size_t(ex) * (p + 1) + a) * (p + 1) + kk] = out[kk];
            }
        }
    }

    // S^0: glue boundary dofs with coinciding Greville anchors
    g->n0 = 0;
    g->s2_to_s0.assign(g->n2, 0);
    if (p >= 1) {
        const int k = g->k;
        std::vector<double> grev(k);
        {
            std::vector<double> kn(size_t(k) + p + 1);
            for (int i = 0; i <= p; ++i) {
                kn[i] = 0.0;
                kn[kn.size() - 1 - i] = 1.0;
            }
            for (int i = 1; i < nel1; ++i) kn[p + i] = double(i) / nel1;
            for (int i = 0; i < k; ++i) {
                double sum = 0;
                for (int r = 1; r <= p; ++r) sum += kn[i + r];
                grev[i] = sum / p;
            }
        }
        std::vector<int> bidx;
        std::vector<double> bpts;
        for (int j = 0; j < npatch; ++j)
            for (int iv = 0; iv < k; ++iv)
                for (int iu = 0; iu < k; ++iu) {
                    if (!(iu == 0 || iu == k - 1 || iv == 0 || iv == k - 1)) continue;
                    double u = grev[iu], v = grev[iv];
                    int ex = std::min(int(u * nel1), nel1 - 1), ey = std::min(int(v * nel1), nel1 - 1);
                    int64_t e = (int64_t(j) * nel1 + ey) * nel1 + ex;
                    double F[3];
                    eval_element_host(g, e, u * nel1 - ex, v * nel1 - ey, F, nullptr, nullptr);
                    bidx.push_back(int((int64_t(j) * k + iv) * k + iu));
                    for (int c = 0; c < 3; ++c) bpts.push_back(F[c]);
                }
        std::vector<int> lab = match_points(bpts, tol);
        // representative = smallest S^2 index of each group
        std::vector<int> rep(g->n2);
        std::iota(rep.begin(), rep.end(), 0);
        std::unordered_map<int, int> grp_min;
        for (size_t i = 0; i < bidx.size(); ++i) {
            auto it = grp_min.find(lab[i]);
            if (it == grp_min.end()) grp_min[lab[i]] = bidx[i];
            else it->second = std::min(it->second, bidx[i]);
        }
        for (size_t i = 0; i < bidx.size(); ++i) rep[bidx[i]] = grp_min[lab[i]];
        std::vector<int> is_rep(g->n2, 0);
        for (int64_t i = 0; i < g->n2; ++i) is_rep[rep[i]] = 1;
        std::vector<int> num(g->n2, -1);
        int n0 = 0;
        for (int64_t i = 0; i < g->n2; ++i)
            if (is_rep[i]) num[i] = n0++;
        for (int64_t i = 0; i < g->n2; ++i) g->s2_to_s0[i] = num[rep[i]];
        g->n0 = n0;
        g->s0_ptr.assign(n0 + 1, 0);
        for (int64_t i = 0; i < g->n2; ++i) g->s0_ptr[g->s2_to_s0[i] + 1]++;
        for (int i = 0; i < n0; ++i) g->s0_ptr[i + 1] += g->s0_ptr[i];
        g->s0_reps.assign(g->n2, 0);
        std::vector<int> fill(g->s0_ptr.begin(), g->s0_ptr.end() - 1);
        for (int64_t i = 0; i < g->n2; ++i) g->s0_reps[fill[g->s2_to_s0[i]]++] = int(i);
    }
    return IGB_OK;
}

}  // namespace igb

// Host side of assemble_nearfield: cluster quadtrees, block partition
// (Sec. 4.4), near element pairs with their quadrature class, and the sparsity
// pattern of the near-field matrix.
#include <algorithm>
#include <array>
#include <cmath>
#include <memory>
#include <map>

#include "common.h"

namespace igb {

void eval_element_host(const igb_geom_s* g, int64_t e, double s, double t, double* F, double* Fs,
                       double* Ft);

namespace {

inline int64_t clu_local(int npatch_unused, int l, int patch, int cx, int cy) {
    (void)npatch_unused;
    return (int64_t(patch) << (2 * l)) + (int64_t(cy) << l) + cx;
}

// square symmetry codes (swap*4 + flip_t*2 + flip_s), acting on local (s,t)
void d4_apply(int code, double s, double t, double& a, double& b) {
    a = s;
    b = t;
    if (code & 4) std::swap(a, b);
    if (code & 1) a = 1.0 - a;
    if (code & 2) b = 1.0 - b;
}

int d4_code(int c0, int c1 /* -1: unused */) {
    // smallest code mapping (0,0) to corner c0 and (1,0) to corner c1
    for (int code = 0; code < 8; ++code) {
        double a, b;
        d4_apply(code, 0, 0, a, b);
        if (int(a) + 2 * int(b) != c0) continue;
        if (c1 >= 0) {
            d4_apply(code, 1, 0, a, b);
            if (int(a) + 2 * int(b) != c1) continue;
        }
        return code;
    }
    return -1;
}

}  // namespace

// Splits every target's far list (pairs sorted by target within a level) into
// chunks of at most `ch` consecutive pairs.
static void build_chunks(igb_op op, int ch, M2LChunks& out) {
    const int np = op->geom->npatch;
    out.tgt.clear();
    out.pair.clear();
    out.len.clear();
    out.tgt_ptr.assign(op->nclusters + 1, 0);
    for (int l = 0; l <= op->L; ++l) {
        const FarLevel& F = op->far[l];
        const int64_t nc = clusters_on_level(np, l);
        for (int64_t t = 0; t < nc; ++t) {
            const int a = F.tgt_ptr[t], b = F.tgt_ptr[t + 1];
            for (int c = a; c < b; c += ch) {
                out.tgt.push_back(int(op->clu_off[l] + t));
                out.pair.push_back(F.pair_off + c);
                out.len.push_back(std::min(ch, b - c));
                out.tgt_ptr[op->clu_off[l] + t + 1]++;
            }
        }
    }
    for (int64_t i = 0; i < op->nclusters; ++i) out.tgt_ptr[i + 1] += out.tgt_ptr[i];
}

igb_status tree_build(igb_op op) {
    igb_geom g = op->geom;
    const int np = g->npatch, m = g->m, nel1 = g->nel1;
    op->d = std::min(std::max(op->prm.leaf_depth, 0), m);
    op->L = m - op->d;
    const int L = op->L;
    op->clu_off.assign(L + 2, 0);
    for (int l = 0; l <= L; ++l) op->clu_off[l + 1] = op->clu_off[l] + clusters_on_level(np, l);
    op->nclusters = op->clu_off[L + 1];
    op->clo.assign(op->nclusters * 3, 0.0);
    op->chi.assign(op->nclusters * 3, 0.0);

    // boxes: elements merged upward level by level; with them the geometry knot
    // span holding the cluster (-1 where its elements lie in several spans)
    std::vector<double> lo(g->lo), hi(g->hi);
    std::vector<int64_t> span(size_t(g->nelem));
    for (int64_t e = 0; e < g->nelem; ++e) span[e] = (int64_t(g->espan[2 * e]) << 32) | g->espan[2 * e + 1];
    std::vector<char> one_span(size_t(op->nclusters), 0);
    for (int l = m; l >= 0; --l) {
        const int n = 1 << l;
        if (l <= L) {
            for (int j = 0; j < np; ++j)
                for (int cy = 0; cy < n; ++cy)
                    for (int cx = 0; cx < n; ++cx) {
                        int64_t src = (int64_t(j) * n + cy) * n + cx;
                        int64_t dst = op->clu_off[l] + clu_local(np, l, j, cx, cy);
                        for (int c = 0; c < 3; ++c) {
                            op->clo[3 * dst + c] = lo[3 * src + c];
                            op->chi[3 * dst + c] = hi[3 * src + c];
                        }
                        one_span[dst] = span[src] >= 0;
                    }
        }
        if (l == 0) break;
        const int h = n / 2;
        std::vector<double> plo(size_t(np) * h * h * 3, 1e300), phi(size_t(np) * h * h * 3, -1e300);
        std::vector<int64_t> pspan(size_t(np) * h * h, -2);   // -2: no child seen yet
        for (int j = 0; j < np; ++j)
            for (int cy = 0; cy < n; ++cy)
                for (int cx = 0; cx < n; ++cx) {
                    int64_t src = (int64_t(j) * n + cy) * n + cx;
                    int64_t dst = (int64_t(j) * h + cy / 2) * h + cx / 2;
                    for (int c = 0; c < 3; ++c) {
                        plo[3 * dst + c] = std::min(plo[3 * dst + c], lo[3 * src + c]);
                        phi[3 * dst + c] = std::max(phi[3 * dst + c], hi[3 * src + c]);
                    }
                    int64_t& ps = pspan[dst];
                    ps = ps == -2 ? span[src] : (ps == span[src] ? ps : -1);
                }
        lo.swap(plo);
        hi.swap(phi);
        span.swap(pspan);
    }
    (void)nel1;

    // A pair is interpolated only where both clusters lie inside one knot span of
    // their patch's geometry: across a knot line a spline mapping is only finitely
    // smooth (the surface measure and normal of a degree-2 mapping have kinks), and
    // the interpolation error of the pulled-back kernel then decays only
    // algebraically in q; inside one span the mapping is one rational piece.
    auto admissible = [&](int64_t t, int64_t s) {
        if (!one_span[t] || !one_span[s]) return false;
        const double *lt = &op->clo[3 * t], *ht = &op->chi[3 * t];
        const double *ls = &op->clo[3 * s], *hs = &op->chi[3 * s];
        double gap2 = 0, dt2 = 0, ds2 = 0;
        for (int c = 0; c < 3; ++c) {
            double gp = std::max(0.0, std::max(ls[c] - ht[c], lt[c] - hs[c]));
            gap2 += gp * gp;
            dt2 += (ht[c] - lt[c]) * (ht[c] - lt[c]);
            ds2 += (hs[c] - ls[c]) * (hs[c] - ls[c]);
        }
        double dm = std::max(std::sqrt(dt2), std::sqrt(ds2));
        if (op->prm.kcap > 0 && op->kappa * dm > op->prm.kcap) return false;
        return std::sqrt(gap2) >= op->prm.eta_adm * dm;
    };

    // level-synchronous dual traversal
    op->far.assign(L + 1, FarLevel());
    std::vector<std::pair<int, int>> cur, nxt;  // local indices on the current level
    for (int a = 0; a < np; ++a)
        for (int b = 0; b < np; ++b) cur.emplace_back(a, b);
    std::vector<std::vector<int>>& near_leaf = op->near_leaf;
    near_leaf.assign(clusters_on_level(np, L), std::vector<int>());
    int64_t pair_off = 0;
    for (int l = 0; l <= L; ++l) {
        const int n = 1 << l;
        std::vector<std::pair<int, int>> farl;
        nxt.clear();
        for (auto& pr : cur) {
            int64_t tg = op->clu_off[l] + pr.first, sg = op->clu_off[l] + pr.second;
            if (admissible(tg, sg)) {
                farl.push_back(pr);
            } else if (l == L) {
                near_leaf[pr.first].push_back(pr.second);
            } else {
                int tj = pr.first >> (2 * l), tr = pr.first & ((1 << (2 * l)) - 1);
                int sj = pr.second >> (2 * l), sr = pr.second & ((1 << (2 * l)) - 1);
                int tcy = tr >> l, tcx = tr & (n - 1), scy = sr >> l, scx = sr & (n - 1);
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) {
                        int tc = int(clu_local(np, l + 1, tj, 2 * tcx + (a & 1), 2 * tcy + (a >> 1)));
                        int sc = int(clu_local(np, l + 1, sj, 2 * scx + (b & 1), 2 * scy + (b >> 1)));
                        nxt.emplace_back(tc, sc);
                    }
            }
        }
        std::sort(farl.begin(), farl.end());
        FarLevel& F = op->far[l];
        F.level = l;
        F.pair_off = pair_off;
        const int64_t nc = clusters_on_level(np, l);
        F.tgt_ptr.assign(nc + 1, 0);
        F.src.resize(farl.size());
        for (size_t i = 0; i < farl.size(); ++i) {
            F.tgt_ptr[farl[i].first + 1]++;
            F.src[i] = farl[i].second;
        }
        for (int64_t i = 0; i < nc; ++i) F.tgt_ptr[i + 1] += F.tgt_ptr[i];
        pair_off += farl.size();
        cur.swap(nxt);
    }
    op->nfar = pair_off;
    op->far_lmin = L + 1;
    for (int l = L; l >= 0; --l)
        if (!op->far[l].src.empty()) op->far_lmin = l;

    // near element pairs, per target element sorted by source element
    const int64_t E = g->nelem;
    const int s = 1 << op->d;   // elements per leaf side
    const int nl = 1 << L;
    op->near_ptr.assign(E + 1, 0);
    for (auto& v : near_leaf) std::sort(v.begin(), v.end());
    for (int64_t e = 0; e < E; ++e) {
        int j = int(e / (int64_t(nel1) * nel1));
        int rem = int(e % (int64_t(nel1) * nel1));
        int ey = rem / nel1, ex = rem % nel1;
        int leaf = int(clu_local(np, L, j, ex / s, ey / s));
        op->near_ptr[e + 1] = op->near_ptr[e] + int64_t(near_leaf[leaf].size()) * s * s;
    }
    op->near_src.resize(op->near_ptr[E]);
    parallel_for(E, 256, [&](int64_t e) {
        int j = int(e / (int64_t(nel1) * nel1));
        int rem = int(e % (int64_t(nel1) * nel1));
        int ey = rem / nel1, ex = rem % nel1;
        int leaf = int(clu_local(np, L, j, ex / s, ey / s));
        int* src = op->near_src.data() + op->near_ptr[e];
        int64_t c = 0;
        for (int sl : near_leaf[leaf]) {
            int sj = sl >> (2 * L), sr = sl & ((1 << (2 * L)) - 1);
            int scy = sr >> L, scx = sr & (nl - 1);
            for (int fy = scy * s; fy < (scy + 1) * s; ++fy)
                for (int fx = scx * s; fx < (scx + 1) * s; ++fx)
                    src[c++] = int((int64_t(sj) * nel1 + fy) * nel1 + fx);
        }
        std::sort(src, src + c);
    });

    // M2L work decompositions: chunks of at most M2L_CHUNK (vector path) and
    // M2L_CHUNK_MFMA (matrix-core path) sources of one target
    build_chunks(op, M2L_CHUNK, op->chunks);
    // (matrix-core chunks shrink, down to 2 sources, until there are about
    // M2L_MFMA_CHUNKS_MIN of them: an operator with few far pairs otherwise
    // leaves most CUs idle in its block products.  Sound-hard chunks start 4x
    // longer: each writes 10 partial vectors, at 16 sources a quarter of the
    // bytes of its bf16 tiles; on the level-7 hard star the partials' reduction
    // went from 2.7 to 0.8 ms and the 16-column product from 36.3 to 33.9 ms.)
    int chm = op->bc == IGB_HARD ? 4 * M2L_CHUNK_MFMA : M2L_CHUNK_MFMA;
    while (chm > 2 && op->nfar / chm < M2L_MFMA_CHUNKS_MIN) chm /= 2;
    build_chunks(op, chm, op->chunks_mfma);
    return IGB_OK;
}

// Gauss order per direction of a regular pair's tensor rule on one element:
// from r = centre distance / (sqrt 2 * the element's extent in that direction),
// so that a square element gets the same order in both directions and an
// element much longer in one direction gets more points along it.
static int regular_order(double r) {
    return r >= 6.0 ? 4 : r >= 3.0 ? 5 : r >= 1.8 ? 6 : r >= 1.2 ? 7 : r >= 0.8 ? 8 : r >= 0.5 ? 10 : 12;
}

// Quadrature class of every near element pair:
//   bits 0..3  : 0 regular, 1 common vertex, 2 common edge, 4 identical
//   regular:  bits 8..11 / 12..15: Gauss orders along u / v on the test element,
//             bits 16..19 / 20..23: the same on the trial element
//   touching: bits 16..18: square symmetry of the test element, 20..22: of the trial element
// Regular orders per direction (regular_order), raised with kappa * diagonal and
// quad_extra, each in [2, 12] and at most REG_POINTS_MAX points per element (the
// shorter direction gives way).
igb_status near_classify(igb_op op) {
    igb_geom g = op->geom;
    const int64_t E = g->nelem;
    std::vector<double> ctr(E * 3), diag(E), side(E * 2);
    for (int64_t e = 0; e < E; ++e) {
        eval_element_host(g, e, 0.5, 0.5, &ctr[3 * e], nullptr, nullptr);
        double a[3], b[3], c[3], d[3], du = 0, dv = 0;
        eval_element_host(g, e, 0.0, 0.5, a, nullptr, nullptr);
        eval_element_host(g, e, 1.0, 0.5, b, nullptr, nullptr);
        eval_element_host(g, e, 0.5, 0.0, c, nullptr, nullptr);
        eval_element_host(g, e, 0.5, 1.0, d, nullptr, nullptr);
        for (int k = 0; k < 3; ++k) {
            du += (b[k] - a[k]) * (b[k] - a[k]);
            dv += (d[k] - c[k]) * (d[k] - c[k]);
        }
        side[2 * e] = std::sqrt(du);
        side[2 * e + 1] = std::sqrt(dv);
        double s2 = 0;
        for (int c = 0; c < 3; ++c) s2 += (g->hi[3 * e + c] - g->lo[3 * e + c]) * (g->hi[3 * e + c] - g->lo[3 * e + c]);
        diag[e] = std::sqrt(s2);
    }
    op->kd_elem = op->kappa * *std::max_element(diag.begin(), diag.end());
    op->aspect_max = 1;
    for (int64_t e = 0; e < E; ++e)
        op->aspect_max = std::max(op->aspect_max, std::max(side[2 * e], side[2 * e + 1]) /
                                                      std::max(1e-300, std::min(side[2 * e], side[2 * e + 1])));
    op->near_kind.resize(op->near_src.size());
    std::atomic<int> bad_shared{-1};   // first inconsistency found: shared corner count (or 2)
    parallel_for(E, 64, [&](int64_t e) {
        for (int64_t k = op->near_ptr[e]; k < op->near_ptr[e + 1]; ++k) {
            const int64_t f = op->near_src[k];
            int shared = 0, ce[4], cf[4];
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    if (g->vert[4 * e + a] == g->vert[4 * f + b]) {
                        ce[shared] = a;
                        cf[shared] = b;
                        ++shared;
                    }
            int kind = 0;
            if (e == f) {
                kind = 4;
            } else if (shared == 2) {
                int te = d4_code(ce[0], ce[1]), tf = d4_code(cf[0], cf[1]);
                if (te < 0 || tf < 0) {
                    int expect = -1;
                    bad_shared.compare_exchange_strong(expect, 2);
                }
                kind = 2 | (te << 16) | (tf << 20);
            } else if (shared == 1) {
                int te = d4_code(ce[0], -1), tf = d4_code(cf[0], -1);
                kind = 1 | (te << 16) | (tf << 20);
            } else if (shared == 0) {
                double d2 = 0;
                for (int c = 0; c < 3; ++c) d2 += (ctr[3 * e + c] - ctr[3 * f + c]) * (ctr[3 * e + c] - ctr[3 * f + c]);
                const double dmax = std::max(diag[e], diag[f]);
                const double dist = std::sqrt(d2);
                // raised with kappa * diameter (oscillation of e^{i kappa r} across the pair)
                const int raise = kd_boost(op->kappa * dmax) + op->prm.quad_extra;
                int ord[4];
                for (int x = 0; x < 2; ++x) {
                    const int64_t el = x ? f : e;
                    int nu = regular_order(dist / (std::sqrt(2.0) * side[2 * el])) + raise;
                    int nv = regular_order(dist / (std::sqrt(2.0) * side[2 * el + 1])) + raise;
                    nu = std::max(2, std::min(nu, 12));
                    nv = std::max(2, std::min(nv, 12));
                    if (nu * nv > REG_POINTS_MAX) {
                        if (nu >= nv)
                            nv = REG_POINTS_MAX / nu;
                        else
                            nu = REG_POINTS_MAX / nv;
                    }
                    ord[2 * x] = nu;
                    ord[2 * x + 1] = nv;
                }
                kind = (ord[0] << 8) | (ord[1] << 12) | (ord[2] << 16) | (ord[3] << 20);
            } else {
                int expect = -1;
                bad_shared.compare_exchange_strong(expect, shared);
            }
            op->near_kind[k] = kind;
        }
    });
    if (bad_shared.load() == 2) {
        set_error("assemble_nearfield: shared edge not on a side of both elements");
        return IGB_ERR_GEOMETRY;
    }
    if (bad_shared.load() >= 0) {
        set_error("assemble_nearfield: elements share %d corners", bad_shared.load());
        return IGB_ERR_GEOMETRY;
    }
    return IGB_OK;
}

// CSR pattern of the near-field matrix in the solution space: column l of row
// r is present iff an element pair (e, f) of the near list has e in the support
// of a representative of r and f in the support of a representative of l.
// Every element of a leaf has the same near sources (the elements of the leaf's
// inadmissible leaves), so a row's columns are the union, over the leaves that
// hold its support, of the columns each leaf's near sources touch.
igb_status near_pattern(igb_op op) {
    igb_geom g = op->geom;
    const int p = g->p, k = g->k, nel1 = g->nel1, np = g->npatch;
    const int L = op->L, s = 1 << op->d, nl = 1 << L;
    const bool hard = op->bc == IGB_HARD;
    const int64_t N = op->N;
    const int64_t nleaf = int64_t(op->near_leaf.size());

    std::vector<std::vector<int>> leaf_cols(nleaf);
    parallel_for(nleaf, 1, [&](int64_t lf) {
        std::vector<int>& c = leaf_cols[lf];
        for (int sl : op->near_leaf[lf]) {
            int sj = sl >> (2 * L), sr = sl & ((1 << (2 * L)) - 1);
            int scy = sr >> L, scx = sr & (nl - 1);
            for (int iy = scy * s; iy < (scy + 1) * s + p; ++iy)
                for (int ix = scx * s; ix < (scx + 1) * s + p; ++ix) {
                    int64_t i2 = (int64_t(sj) * k + iy) * k + ix;
                    c.push_back(int(hard ? g->s2_to_s0[i2] : i2));
                }
        }
        std::sort(c.begin(), c.end());
        c.erase(std::unique(c.begin(), c.end()), c.end());
    });

    // leaves holding the support of row r (sorted, unique)
    auto row_leaves = [&](int64_t r, std::vector<int>& out) {
        out.clear();
        auto add_rep = [&](int64_t i) {
            int j = int(i / (int64_t(k) * k));
            int rem = int(i % (int64_t(k) * k));
            int iv = rem / k, iu = rem % k;
            int y0 = std::max(0, iv - p) / s, y1 = std::min(iv, nel1 - 1) / s;
            int x0 = std::max(0, iu - p) / s, x1 = std::min(iu, nel1 - 1) / s;
            for (int ly = y0; ly <= y1; ++ly)
                for (int lx = x0; lx <= x1; ++lx) out.push_back(int(clu_local(np, L, j, lx, ly)));
        };
        if (hard) {
            for (int q = g->s0_ptr[r]; q < g->s0_ptr[r + 1]; ++q) add_rep(g->s0_reps[q]);
        } else {
            add_rep(r);
        }
        std::sort(out.begin(), out.end());
        out.erase(std::unique(out.begin(), out.end()), out.end());
    };
    // union of the leaves' column lists into `buf` (returns its length)
    auto merge = [&](const std::vector<int>& leaves, std::vector<int>& buf, std::vector<int>& tmp) {
        buf.assign(leaf_cols[leaves[0]].begin(), leaf_cols[leaves[0]].end());
        for (size_t i = 1; i < leaves.size(); ++i) {
            const std::vector<int>& c = leaf_cols[leaves[i]];
            tmp.resize(buf.size() + c.size());
            auto end = std::set_union(buf.begin(), buf.end(), c.begin(), c.end(), tmp.begin());
            tmp.resize(end - tmp.begin());
            buf.swap(tmp);
        }
    };

    op->row_ptr.assign(N + 1, 0);
    parallel_for(N, 256, [&](int64_t r) {
        thread_local std::vector<int> leaves, buf, tmp;
        row_leaves(r, leaves);
        if (leaves.size() == 1) {
            op->row_ptr[r + 1] = int64_t(leaf_cols[leaves[0]].size());
        } else {
            merge(leaves, buf, tmp);
            op->row_ptr[r + 1] = int64_t(buf.size());
        }
    });
    for (int64_t r = 0; r < N; ++r) op->row_ptr[r + 1] += op->row_ptr[r];
    op->nnz = op->row_ptr[N];
    op->col.resize(op->nnz);
    parallel_for(N, 256, [&](int64_t r) {
        thread_local std::vector<int> leaves, buf, tmp;
        row_leaves(r, leaves);
        const std::vector<int>* src = &leaf_cols[leaves[0]];
        if (leaves.size() > 1) {
            merge(leaves, buf, tmp);
            src = &buf;
        }
        std::copy(src->begin(), src->end(), op->col.begin() + op->row_ptr[r]);
    });

    // rows with the same leaves (hence the same column list) form
    // groups, taken in order of their first row; up to 16 rows of neighbouring
    // groups share a tile whose columns are the union of theirs, as long as the
    // union stays within NEAR_TILE_FILL of the longest member list (the rows'
    // missing columns are stored as zeros; fewer, fuller tiles gather x less often)
    op->near_tiles.clear();
    op->near_tile_cols.clear();
    op->near_tile_vals = 0;
    std::map<std::vector<int>, std::vector<int>> groups;
    {
        std::vector<int> leaves;
        for (int64_t r = 0; r < N; ++r) {
            row_leaves(r, leaves);
            groups[leaves].push_back(int(r));
        }
    }
    std::vector<const std::vector<int>*> order;
    for (const auto& kv : groups) order.push_back(&kv.second);
    std::sort(order.begin(), order.end(),
              [](const std::vector<int>* a, const std::vector<int>* b) { return a->front() < b->front(); });
    // each group's column list once; every row points at its group's list
    op->near_dcol.clear();
    op->row_coff.assign(N, 0);
    op->near_wgs.clear();
    op->near_grp_rows.clear();
    op->near_list_max = 0;
    for (const std::vector<int>* g : order) {
        const int64_t off = int64_t(op->near_dcol.size());
        const int len = int(op->row_ptr[g->front() + 1] - op->row_ptr[g->front()]);
        op->near_dcol.insert(op->near_dcol.end(), op->col.begin() + op->row_ptr[g->front()],
                             op->col.begin() + op->row_ptr[g->front() + 1]);
        op->near_list_max = std::max(op->near_list_max, len);
        for (size_t i = 0; i < g->size(); i += NEAR_GROUP_ROWS) {
            NearGroupWG w{};
            w.list_off = off;
            w.list_len = len;
            w.row0 = int(op->near_grp_rows.size() + i);
            w.nrows = int(std::min<size_t>(NEAR_GROUP_ROWS, g->size() - i));
            op->near_wgs.push_back(w);
        }
        for (int r : *g) {
            op->row_coff[r] = off;
            op->near_grp_rows.push_back(r);
        }
    }
    {
        // bf16 operators use the tiles with fp32 values (inner matvecs), fp64
        // operators with fp64 values (blocks of >= 16 columns); built for every
        // operator (host plan only)
        std::vector<int> rows, cols, tmp;
        size_t longest = 0;
        auto emit = [&]() {
            if (rows.empty()) return;
            NearTile t{};
            t.val_off = op->near_tile_vals;
            t.col_off = int64_t(op->near_tile_cols.size());
            t.ncols = int(cols.size());
            t.nrows = int(rows.size());
            for (int i = 0; i < NEAR_TILE_ROWS; ++i) t.rows[i] = i < t.nrows ? rows[i] : -1;
            op->near_tile_cols.insert(op->near_tile_cols.end(), cols.begin(), cols.end());
            op->near_tile_vals += int64_t((t.ncols + NEAR_TILE_K - 1) / NEAR_TILE_K) * t.nrows * NEAR_TILE_K;
            op->near_tiles.push_back(t);
            rows.clear();
            cols.clear();
            longest = 0;
        };
        for (const std::vector<int>* g : order) {
            const int* c0 = op->col.data() + op->row_ptr[g->front()];
            const size_t nc = size_t(op->row_ptr[g->front() + 1] - op->row_ptr[g->front()]);
            for (size_t i0 = 0; i0 < g->size(); i0 += NEAR_TILE_ROWS) {
                const size_t nr = std::min<size_t>(NEAR_TILE_ROWS, g->size() - i0);
                if (!rows.empty()) {
                    tmp.resize(cols.size() + nc);
                    tmp.resize(std::set_union(cols.begin(), cols.end(), c0, c0 + nc, tmp.begin()) - tmp.begin());
                    const size_t lim = size_t(double(std::max(longest, nc)) * (1.0 + NEAR_TILE_FILL));
                    if (rows.size() + nr <= size_t(NEAR_TILE_ROWS) && tmp.size() <= lim) {
                        cols.swap(tmp);
                    } else {
                        emit();
                    }
                }
                if (rows.empty()) cols.assign(c0, c0 + nc);
                rows.insert(rows.end(), g->begin() + i0, g->begin() + i0 + nr);
                longest = std::max(longest, nc);
            }
        }
        emit();
    }
    return IGB_OK;
}


// --------------------------------------------------------------------------
// Target boxes and interaction lists of the H^2 potential evaluation
// --------------------------------------------------------------------------
igb_status potential_plan(igb_op op, const double* pts, int npts, PotentialPlan& P) {
    igb_geom g = op->geom;
    const int np = g->npatch, m = g->m, L = std::max(m - 1, 0);
    // source cluster boxes, levels 0..L: the elements' boxes merged upward
    P.lmax = L;
    P.off.assign(L + 2, 0);
    for (int l = 0; l <= L; ++l) P.off[l + 1] = P.off[l] + clusters_on_level(np, l);
    std::vector<double> clo(size_t(P.off[L + 1]) * 3), chi(size_t(P.off[L + 1]) * 3);
    {
        std::vector<double> lo(g->lo), hi(g->hi);
        for (int l = m; l >= 0; --l) {
            const int n = 1 << l;
            if (l <= L)
                for (int64_t src = 0; src < clusters_on_level(np, l); ++src)
                    for (int c = 0; c < 3; ++c) {
                        clo[3 * (P.off[l] + src) + c] = lo[3 * src + c];
                        chi[3 * (P.off[l] + src) + c] = hi[3 * src + c];
                    }
            if (l == 0) break;
            const int h = n / 2;
            std::vector<double> plo(size_t(np) * h * h * 3, 1e300), phi(size_t(np) * h * h * 3, -1e300);
            for (int j = 0; j < np; ++j)
                for (int cy = 0; cy < n; ++cy)
                    for (int cx = 0; cx < n; ++cx) {
                        const int64_t src = (int64_t(j) * n + cy) * n + cx;
                        const int64_t dst = (int64_t(j) * h + cy / 2) * h + cx / 2;
                        for (int c = 0; c < 3; ++c) {
                            plo[3 * dst + c] = std::min(plo[3 * dst + c], lo[3 * src + c]);
                            phi[3 * dst + c] = std::max(phi[3 * dst + c], hi[3 * src + c]);
                        }
                    }
            lo.swap(plo);
            hi.swap(phi);
        }
    }
    P.perm.resize(npts);
    for (int i = 0; i < npts; ++i) P.perm[i] = i;
    P.box_ptr.assign(1, 0);
    P.box_lo.clear();
    P.box_hi.clear();
    if (npts == 0) {
        P.far_ptr.assign(1, 0);
        P.m2p_ptr.assign(1, 0);
        P.near_ptr.assign(1, 0);
        P.far_src.clear();
        P.m2p_src.clear();
        P.near_leaf.clear();
        return IGB_OK;
    }
    double glo[3], ghi[3];
    for (int c = 0; c < 3; ++c) glo[c] = ghi[c] = pts[c];
    for (int i = 0; i < npts; ++i)
        for (int c = 0; c < 3; ++c) {
            glo[c] = std::min(glo[c], pts[3 * i + c]);
            ghi[c] = std::max(ghi[c], pts[3 * i + c]);
        }
    double side = 0;
    for (int c = 0; c < 3; ++c) side = std::max(side, ghi[c] - glo[c]);
    if (!(side > 0)) side = 1.0;
    // A cluster is interpolated only if it spans at most kcap radians of e^{i kappa r}
    // (the operator's kcap, else q / 2: q + 1 Chebyshev points per direction), and so
    // is the box where its points share the box's nodes.  (A cap of q - 1 on the
    // cluster alone was 1.3-6x faster on the level-5 sphere at kappa = 8, but its
    // error against the direct sum rose from 7e-9 to 2e-6.)
    const double kcap = op->prm.kcap > 0 ? op->prm.kcap : 0.5 * op->q;
    const int64_t n3 = int64_t(op->q + 1) * (op->q + 1) * (op->q + 1);
    // octree of cubes over index ranges, leaves (the interpolation boxes) in
    // depth-first octant order; the coordinates travel with the permutation so
    // that every pass reads them in order
    struct Node {
        int b, e, depth;
        double lo[3], h;
    };
    // (smaller boxes at high kappa, so that more of them can interpolate, cost
    // more per point on the m = 5 sphere at kappa = 8 than they save)
    const auto is_leaf = [](const Node& nd) { return nd.e - nd.b <= POT_LEAF_POINTS || nd.depth >= 20; };
    // work arrays left uninitialised and first touched by the threads that use them
    std::unique_ptr<double[]> xs(new double[3 * size_t(npts)]), xtmp(new double[3 * size_t(npts)]);
    std::unique_ptr<int[]> ptmp(new int[npts]);
    std::unique_ptr<unsigned char[]> code(new unsigned char[npts]);
    constexpr int64_t GRAIN = 1 << 16;
    parallel_for((npts + GRAIN - 1) / GRAIN, 1, [&](int64_t k) {
        const int64_t a = k * GRAIN, e = std::min<int64_t>(npts, a + GRAIN);
        std::copy(pts + 3 * a, pts + 3 * e, xs.get() + 3 * a);
    });
    // stable partition of [b, e) into the 8 octants, in chunks of GRAIN points (the
    // chunks in parallel when wide); the non-empty children in octant order
    const auto split = [&](const Node& nd, bool wide, std::vector<Node>& kids) {
        const double h = 0.5 * nd.h;
        const int64_t nch = (nd.e - nd.b + GRAIN - 1) / GRAIN;
        std::vector<std::array<int, 8>> cnt(nch);
        const auto over = [&](const auto& f) {
            if (wide) parallel_for(nch, 1, f);
            else for (int64_t k = 0; k < nch; ++k) f(k);
        };
        over([&](int64_t k) {
            cnt[k].fill(0);
            const int a = nd.b + int(k * GRAIN), e = std::min<int64_t>(nd.e, a + GRAIN);
            for (int i = a; i < e; ++i) {
                int o = 0;
                for (int c = 0; c < 3; ++c)
                    if (xs[3 * size_t(i) + c] >= nd.lo[c] + h) o |= 1 << c;
                code[i] = (unsigned char)o;
                ++cnt[k][o];
            }
        });
        // chunk k's points of octant o start after all points of lower octants and
        // after the octant-o points of chunks before k
        int start[9];
        start[0] = nd.b;
        for (int o = 0; o < 8; ++o) {
            int tot = 0;
            for (int64_t k = 0; k < nch; ++k) tot += cnt[k][o];
            start[o + 1] = start[o] + tot;
        }
        std::vector<std::array<int, 8>> pos(nch);
        for (int o = 0; o < 8; ++o) {
            int p = start[o];
            for (int64_t k = 0; k < nch; ++k) {
                pos[k][o] = p;
                p += cnt[k][o];
            }
        }
        over([&](int64_t k) {
            const int a = nd.b + int(k * GRAIN), e = std::min<int64_t>(nd.e, a + GRAIN);
            for (int i = a; i < e; ++i) {
                const size_t j = size_t(pos[k][code[i]]++);
                ptmp[j] = P.perm[i];
                for (int c = 0; c < 3; ++c) xtmp[3 * j + c] = xs[3 * size_t(i) + c];
            }
        });
        over([&](int64_t k) {
            const int a = nd.b + int(k * GRAIN), e = std::min<int64_t>(nd.e, a + GRAIN);
            std::copy(ptmp.get() + a, ptmp.get() + e, P.perm.begin() + a);
            std::copy(xtmp.get() + 3 * size_t(a), xtmp.get() + 3 * size_t(e), xs.get() + 3 * size_t(a));
        });
        for (int o = 0; o < 8; ++o)
            if (start[o + 1] > start[o])
                kids.push_back(Node{start[o], start[o + 1], nd.depth + 1,
                                    {nd.lo[0] + ((o & 1) ? h : 0), nd.lo[1] + ((o & 2) ? h : 0),
                                     nd.lo[2] + ((o & 4) ? h : 0)},
                                    h});
    };
    // the top levels split level by level into a frontier in depth-first order (a
    // level of few nodes splits each node in parallel, a wider one its nodes in
    // parallel), whose subtrees are then built in parallel
    std::vector<Node> front{Node{0, npts, 0, {glo[0], glo[1], glo[2]}, side}};
    const size_t nthr = size_t(host_threads()), want = 8 * nthr;
    while (front.size() < want && std::any_of(front.begin(), front.end(), [&](const Node& nd) { return !is_leaf(nd); })) {
        std::vector<std::vector<Node>> kids(front.size());
        const auto one = [&](int64_t f, bool wide) {
            if (is_leaf(front[f])) kids[f].push_back(front[f]);
            else split(front[f], wide, kids[f]);
        };
        if (front.size() < nthr)
            for (size_t f = 0; f < front.size(); ++f) one(int64_t(f), true);
        else
            parallel_for(int64_t(front.size()), 1, [&](int64_t f) { one(f, false); });
        std::vector<Node> next;
        for (const auto& k : kids) next.insert(next.end(), k.begin(), k.end());
        front.swap(next);
    }
    struct Leaves {
        std::vector<int> end;
        std::vector<double> lo, hi;
    };
    std::vector<Leaves> sub(front.size());
    parallel_for(int64_t(front.size()), 1, [&](int64_t f) {
        Leaves& out = sub[f];
        std::vector<Node> stack{front[f]}, kids;
        while (!stack.empty()) {
            const Node nd = stack.back();
            stack.pop_back();
            if (!is_leaf(nd)) {
                kids.clear();
                split(nd, false, kids);
                stack.insert(stack.end(), kids.rbegin(), kids.rend());   // octant 0 taken first
                continue;
            }
            // interpolation box: the points' own box, each side at least 1e-3 of the cube
            double lo[3], hi[3];
            for (int c = 0; c < 3; ++c) {
                lo[c] = 1e300;
                hi[c] = -1e300;
            }
            for (int i = nd.b; i < nd.e; ++i)
                for (int c = 0; c < 3; ++c) {
                    lo[c] = std::min(lo[c], xs[3 * size_t(i) + c]);
                    hi[c] = std::max(hi[c], xs[3 * size_t(i) + c]);
                }
            for (int c = 0; c < 3; ++c) {
                const double mid = 0.5 * (lo[c] + hi[c]), half = std::max(0.5 * (hi[c] - lo[c]), 5e-4 * nd.h);
                out.lo.push_back(mid - half);
                out.hi.push_back(mid + half);
            }
            out.end.push_back(nd.e);
        }
    });
    for (const auto& s : sub) {
        P.box_ptr.insert(P.box_ptr.end(), s.end.begin(), s.end.end());
        P.box_lo.insert(P.box_lo.end(), s.lo.begin(), s.lo.end());
        P.box_hi.insert(P.box_hi.end(), s.hi.begin(), s.hi.end());
    }
    const int64_t nbox = int64_t(P.box_ptr.size()) - 1;
    // interaction lists: descend the source cluster tree from the patches
    std::vector<std::vector<int>> far(nbox), m2p(nbox), near(nbox);
    parallel_for(nbox, 16, [&](int64_t b) {
        const double* lt = &P.box_lo[3 * b];
        const double* ht = &P.box_hi[3 * b];
        // interpolating on the box pays only where it holds more points than nodes
        const bool box_nodes = P.box_ptr[b + 1] - P.box_ptr[b] > n3;
        double dt2 = 0;
        for (int c = 0; c < 3; ++c) dt2 += (ht[c] - lt[c]) * (ht[c] - lt[c]);
        std::vector<std::pair<int, int64_t>> st;   // (level, index on the level)
        for (int j = 0; j < np; ++j) st.push_back({0, j});
        while (!st.empty()) {
            const int l = st.back().first;
            const int64_t loc = st.back().second;
            st.pop_back();
            const int64_t gid = P.off[l] + loc;
            const double *ls = &clo[3 * gid], *hs = &chi[3 * gid];
            double gap2 = 0, ds2 = 0;
            for (int c = 0; c < 3; ++c) {
                const double gp = std::max(0.0, std::max(ls[c] - ht[c], lt[c] - hs[c]));
                gap2 += gp * gp;
                ds2 += (hs[c] - ls[c]) * (hs[c] - ls[c]);
            }
            const double gap = std::sqrt(gap2), ds = std::sqrt(ds2), dm = std::max(std::sqrt(dt2), ds);
            if (box_nodes && gap >= op->prm.eta_adm * dm && op->kappa * dm <= kcap) {
                far[b].push_back(int(gid));
            } else if (gap >= op->prm.eta_adm * ds && op->kappa * ds <= kcap) {
                m2p[b].push_back(int(gid));
            } else if (l == L) {
                near[b].push_back(int(loc));
            } else {
                const int n = 1 << l;
                const int64_t j = loc >> (2 * l);
                const int cy = int((loc >> l) & (n - 1)), cx = int(loc & (n - 1));
                for (int a = 3; a >= 0; --a)
                    st.push_back({l + 1, clu_local(np, l + 1, int(j), 2 * cx + (a & 1), 2 * cy + (a >> 1))});
            }
        }
    });
    P.far_ptr.assign(nbox + 1, 0);
    P.m2p_ptr.assign(nbox + 1, 0);
    P.near_ptr.assign(nbox + 1, 0);
    int64_t tot[3] = {0, 0, 0};
    for (int64_t b = 0; b < nbox; ++b) {
        tot[0] += int64_t(far[b].size());
        tot[1] += int64_t(m2p[b].size());
        tot[2] += int64_t(near[b].size());
    }
    if (std::max(tot[0], std::max(tot[1], tot[2])) > int64_t(INT32_MAX)) {
        set_error("potential_h2: interaction lists of %d points exceed 2^31 entries; pass fewer points per call",
                  npts);
        return IGB_ERR_ARG;
    }
    for (int64_t b = 0; b < nbox; ++b) {
        P.far_ptr[b + 1] = P.far_ptr[b] + int(far[b].size());
        P.m2p_ptr[b + 1] = P.m2p_ptr[b] + int(m2p[b].size());
        P.near_ptr[b + 1] = P.near_ptr[b] + int(near[b].size());
    }
    P.far_src.resize(P.far_ptr[nbox]);
    P.m2p_src.resize(P.m2p_ptr[nbox]);
    P.near_leaf.resize(P.near_ptr[nbox]);
    parallel_for(nbox, 256, [&](int64_t b) {
        std::copy(far[b].begin(), far[b].end(), P.far_src.begin() + P.far_ptr[b]);
        std::copy(m2p[b].begin(), m2p[b].end(), P.m2p_src.begin() + P.m2p_ptr[b]);
        std::copy(near[b].begin(), near[b].end(), P.near_leaf.begin() + P.near_ptr[b]);
        std::vector<int>().swap(far[b]);
        std::vector<int>().swap(m2p[b]);
        std::vector<int>().swap(near[b]);
    });
    return IGB_OK;
}

}  // namespace igb

// Host stages of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
// (built by tests/test_host_sanitizers.py with the sanitizers on the host
// compilation only): geometries at levels 1-4 and degrees 1-3, operators for
// both boundary conditions and all three precisions on a host-only context
// (cluster trees, block partitions, near pairs, CSR patterns, tiles), their
// inspection entry points (the H^2 potential's plan for scattered and repeated
// points among them), the solve size model, a solve refused by the
// host-only context, and every handle destroyed.  Reads the patches from the
// binary file named by argv[1]: int npatch, then per patch int deg_u, deg_v,
// ncp_u, ncp_v, the two knot vectors and the control net (doubles).
#include <cstdio>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <vector>
#include "igafmm.h"
int main(int argc, char** argv) {
    if (argc < 2) return 3;
    std::FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 3;
    int np; std::fread(&np, 4, 1, f);
    std::vector<igb_patch> P(np);
    std::vector<std::vector<double>> ku(np), kv(np), cp(np);
    for (int i = 0; i < np; ++i) {
        int h[4]; std::fread(h, 4, 4, f);
        P[i].deg_u = h[0]; P[i].deg_v = h[1]; P[i].ncp_u = h[2]; P[i].ncp_v = h[3];
        ku[i].resize(h[2] + h[0] + 1); kv[i].resize(h[3] + h[1] + 1); cp[i].resize(size_t(h[2]) * h[3] * 4);
        std::fread(ku[i].data(), 8, ku[i].size(), f); std::fread(kv[i].data(), 8, kv[i].size(), f);
        std::fread(cp[i].data(), 8, cp[i].size(), f);
        P[i].knots_u = ku[i].data(); P[i].knots_v = kv[i].data(); P[i].cpw = cp[i].data();
    }
    std::fclose(f);
    igb_ctx c; if (igb_ctx_create(IGB_HOST_ONLY, 0, &c)) return 1;
    for (int m = 1; m <= 4; ++m) for (int p = 1; p <= 3; ++p) {
        igb_geom g; if (build_geometry(c, P.data(), np, m, p, &g)) { std::printf("geom fail %s\n", igb_last_error()); return 1; }
        for (int bc = 0; bc < 2; ++bc) for (int prec = 0; prec < 3; ++prec) {
            igb_op_params prm{}; prm.kappa = 2.0; prm.bc = bc; prm.q = 4; prm.eta_adm = 1.6; prm.leaf_depth = 1;
            prm.precision = prec; prm.kcap = m == 3 ? 3.0 : 0.0; prm.separate = (m == 2 && prec == 0);
            igb_op op; if (assemble_nearfield(c, g, &prm, &op)) { std::printf("op fail %s\n", igb_last_error()); return 1; }
            igb_op_info info; igb_op_get_info(op, &info);
            int64_t b; igb_op_solve_bytes(op, 16, 30, &b);
            if (!prm.separate) {
                std::vector<int64_t> ptr(info.nelem + 1); std::vector<int32_t> src(info.near_elem_pairs), kind(info.near_elem_pairs);
                igb_op_near_pairs(op, ptr.data(), src.data(), kind.data());
                std::vector<int32_t> fb(4 * info.far_pairs + 4); igb_op_far_blocks(op, fb.data());
            }
            {   // the potential's plan: seeded points in [-3, 3]^3, the last 300 repeated
                const int npt = (m == 2 && bc == 0 && prec == 0) ? 140000 : 2000;
                std::vector<double> x(3 * size_t(npt));
                uint64_t st = 12345u + uint64_t(m) * 7u + uint64_t(p);
                for (auto& v : x) { st = st * 6364136223846793005ull + 1442695040888963407ull; v = 6.0 * double(st >> 11) / 9007199254740992.0 - 3.0; }
                for (int i = npt - 300; i < npt; ++i) for (int c = 0; c < 3; ++c) x[3 * size_t(i) + c] = 2.5;
                int64_t cnt[4];
                if (igb_op_potential_plan(op, x.data(), npt, cnt, nullptr, nullptr)) { std::printf("plan fail %s\n", igb_last_error()); return 1; }
                std::vector<int32_t> perm(npt), bptr(cnt[0] + 1), seen(npt, 0);
                if (igb_op_potential_plan(op, x.data(), npt, cnt, perm.data(), bptr.data())) return 1;
                for (int32_t v : perm) if (v < 0 || v >= npt || seen[v]++) return 4;
                if (bptr[0] != 0 || bptr[cnt[0]] != npt) return 4;
                for (int64_t b = 0; b < cnt[0]; ++b) if (bptr[b + 1] <= bptr[b]) return 4;
                x[7] = std::nan("");
                if (igb_op_potential_plan(op, x.data(), npt, cnt, nullptr, nullptr) != IGB_ERR_ARG) return 2;
            }
            double d[3] = {0, 0, 1}; igb_solve_params sp{1e-8, 30, 10, 0, 0, 0}; igb_solve_info si;
            if (cfie_solve(op, d, 1, &sp, reinterpret_cast<double*>(16), &si) != IGB_ERR_ARG) return 2;
            std::printf("m=%d p=%d bc=%d prec=%d n=%lld far=%lld nnz=%lld model16=%lld\n", m, p, bc, prec,
                        (long long)info.n, (long long)info.far_pairs, (long long)info.nnz, (long long)b);
            igb_op_destroy(op);
        }
        igb_geom_destroy(g);
    }
    igb_ctx_destroy(c);
    std::printf("ok\n");
    return 0;
}

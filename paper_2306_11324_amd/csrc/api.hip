// The C ABI of igafmm (declared in include/igafmm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "common.h"

namespace igb {
const char* last_error();

igb_ctx_s*& alloc_ctx() {
    thread_local igb_ctx_s* c = nullptr;
    return c;
}

bool charge(igb_ctx_s* c, size_t bytes) {
    size_t cur = c->used.load();
    do {
        if (c->budget != 0 && cur + bytes > c->budget) return false;
    } while (!c->used.compare_exchange_weak(cur, cur + bytes));
    return true;
}

igb_status dev_malloc(DevBuf& b, size_t bytes, const char* who) {
    b.release();
    if (bytes == 0) return IGB_OK;
    igb_ctx_s* c = alloc_ctx();
    if (c && !charge(c, bytes)) {
        set_error("%s: HBM budget exceeded (%zu held + %zu > %zu bytes)", who, c->used.load(), bytes, c->budget);
        return IGB_ERR_BUDGET;
    }
    const hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        if (c) uncharge(c, bytes);
        b.ptr = nullptr;
        set_error("%s: hipMalloc of %zu bytes: %s", who, bytes, hipGetErrorString(e));
        return IGB_ERR_HIP;
    }
    b.bytes = bytes;
    b.ctx = c;
    return IGB_OK;
}
}

using namespace igb;

namespace {

hipStream_t pick(igb_ctx ctx, void* s) { return s == IGB_CONTEXT_STREAM ? ctx->stream : static_cast<hipStream_t>(s); }

bool host_only(igb_ctx ctx) { return ctx->device == IGB_HOST_ONLY; }

igb_status need_device(igb_op op, const char* what) {
    if (host_only(op->geom->ctx)) {
        set_error("%s: the operator belongs to a host-only context", what);
        return IGB_ERR_ARG;
    }
    return IGB_OK;
}

// entry points that need a right-hand side / representation (not single operators)
static igb_status need_system(igb_op op, const char* what) {
    if (!op->system) {
        set_error("%s: the operator is a single boundary integral operator (IGB_OP_*), not a system", what);
        return IGB_ERR_ARG;
    }
    return IGB_OK;
}

// entry points that read one H^2 matrix's internals
static igb_status need_single_matrix(igb_op op, const char* what) {
    if (!op->sum_parts.empty()) {
        set_error("%s: not available on an operator stored as separate H^2 matrices", what);
        return IGB_ERR_ARG;
    }
    return IGB_OK;
}

// device bytes held by an operator (its parts, for a lazy sum)
size_t op_held_bytes(igb_op op) {
    size_t b = op->dev_bytes;
    for (igb_op p : op->sum_parts) b += p->dev_bytes;
    return b;
}

bool budget_ok(igb_ctx ctx, size_t add) {
    return ctx->budget == 0 || ctx->used.load() + add <= ctx->budget;
}

}  // namespace

extern "C" {

const char* igb_last_error(void) { return igb::last_error(); }

igb_status igb_ctx_create(int device, size_t hbm_budget_bytes, igb_ctx* out) {
    if (!out) {
        set_error("igb_ctx_create: out is NULL");
        return IGB_ERR_ARG;
    }
    if (device == IGB_HOST_ONLY) {
        igb_ctx c = new (std::nothrow) igb_ctx_s();
        if (!c) {
            set_error("igb_ctx_create: out of host memory");
            return IGB_ERR_ARG;
        }
        c->device = IGB_HOST_ONLY;
        c->budget = hbm_budget_bytes;
        *out = c;
        return IGB_OK;
    }
    int n = 0;
    IGB_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) {
        set_error("igb_ctx_create: device %d out of range (%d devices)", device, n);
        return IGB_ERR_ARG;
    }
    IGB_HIP(hipSetDevice(device));
    igb_ctx c = new (std::nothrow) igb_ctx_s();
    if (!c) {
        set_error("igb_ctx_create: out of host memory");
        return IGB_ERR_ARG;
    }
    c->device = device;
    c->budget = hbm_budget_bytes;
    // locate this device's matvec scratch array (h2_matvec_noalloc) once
    if (igb_status st = scratch_init(device)) {
        delete c;
        return st;
    }
    hipError_t e = hipDeviceGetAttribute(&c->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        set_error("igb_ctx_create: %s", hipGetErrorString(e));
        return IGB_ERR_HIP;
    }
    *out = c;
    return IGB_OK;
}

// Handles are reference counted so that the caller may destroy them in any
// order: a geometry keeps its context alive, an operator its geometry.
void ctx_release(igb_ctx ctx) {
    if (!ctx || --ctx->refs > 0) return;
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

void geom_release(igb_geom g) {
    if (!g || --g->refs > 0) return;
    igb_ctx ctx = g->ctx;
    delete g;
    ctx_release(ctx);
}

void igb_ctx_destroy(igb_ctx ctx) { ctx_release(ctx); }

size_t igb_ctx_used_bytes(igb_ctx ctx) { return ctx ? ctx->used.load() : 0; }

igb_status build_geometry(igb_ctx ctx, const igb_patch* patches, int npatch, int level_m, int degree_p,
                          igb_geom* out) {
    if (!ctx || !patches || !out) {
        set_error("build_geometry: NULL argument");
        return IGB_ERR_ARG;
    }
    AllocScope scope(ctx);
    if (!host_only(ctx)) IGB_HIP(hipSetDevice(ctx->device));
    igb_geom g = new (std::nothrow) igb_geom_s();
    if (!g) {
        set_error("build_geometry: out of host memory");
        return IGB_ERR_ARG;
    }
    igb_status st = geometry_build(ctx, patches, npatch, level_m, degree_p, g);
    if (st) {
        delete g;
        return st;
    }
    const size_t need = g->bez.size() * 8 + g->pg.size() * 4 + g->C1.size() * 8;
    if (!budget_ok(ctx, need)) {
        delete g;
        set_error("build_geometry: HBM budget exceeded (%zu + %zu > %zu bytes)", ctx->used.load(), need, ctx->budget);
        return IGB_ERR_BUDGET;
    }
    if (!host_only(ctx) && (st = upload_geometry(g))) {
        delete g;
        return st;
    }
    ++ctx->refs;
    *out = g;
    return IGB_OK;
}

void igb_geom_destroy(igb_geom g) { geom_release(g); }

igb_status igb_geom_dims(igb_geom g, int64_t dims[3]) {
    if (!g || !dims) {
        set_error("igb_geom_dims: NULL argument");
        return IGB_ERR_ARG;
    }
    dims[0] = g->nelem;
    dims[1] = g->n2;
    dims[2] = g->n0;
    return IGB_OK;
}

// Coefficients of one assembled operator (see the system in igb_op_s)
struct Coefs {
    int family;
    double eta;
    SoftMix mix;
    HardMix hmix;
    double2 cm, rn, rd;
    bool system;   // a right-hand side and a representation exist (not for single operators)
};

static Coefs coefs_for(const igb_op_params* prm) {
    Coefs c{};
    c.system = true;
    c.hmix = HardMix{make_double2(0, 0), make_double2(0, 0)};
    c.mix = SoftMix{0.0, make_double2(0, 0)};
    c.cm = c.rn = c.rd = make_double2(0, 0);
    const bool soft = prm->bc == IGB_SOFT;
    switch (prm->formulation) {
        case IGB_SINGLE_LAYER:
            // u_s = -S t on S^2: V t = u_inc (soft), (K* - 1/2) t = d_n u_inc (hard)
            c.family = IGB_SOFT;
            c.mix = SoftMix{soft ? 0.0 : 1.0, make_double2(soft ? 1.0 : 0.0, 0.0)};
            c.cm = make_double2(soft ? 0.0 : -0.5, 0.0);
            c.rn = make_double2(soft ? 0.0 : 1.0, 0.0);
            c.rd = make_double2(soft ? 1.0 : 0.0, 0.0);
            break;
        case IGB_OP_V:
        case IGB_OP_KSTAR:
            c.family = IGB_SOFT;
            c.mix = SoftMix{prm->formulation == IGB_OP_KSTAR ? 1.0 : 0.0,
                            make_double2(prm->formulation == IGB_OP_V ? 1.0 : 0.0, 0.0)};
            c.system = false;
            break;
        case IGB_OP_K:
        case IGB_OP_W:
            c.family = IGB_HARD;
            c.hmix = HardMix{make_double2(prm->formulation == IGB_OP_K ? 1.0 : 0.0, 0.0),
                             make_double2(prm->formulation == IGB_OP_W ? 1.0 : 0.0, 0.0)};
            c.system = false;
            break;
        default:  // IGB_CFIE
            c.family = prm->bc;
            c.eta = prm->eta_c != 0 ? prm->eta_c : (soft ? prm->kappa : -1.0 / prm->kappa);
            c.cm = make_double2(0.5, 0.0);
            if (soft) {
                // (1/2 M + K* - i eta V) t = <d_n u_inc - i eta u_inc, psi>
                c.mix = SoftMix{1.0, make_double2(0.0, -c.eta)};
                c.rn = make_double2(1.0, 0.0);
                c.rd = make_double2(0.0, -c.eta);
            } else {
                // (1/2 M - K - i eta W) g = <u_inc - i eta d_n u_inc, psi>
                c.hmix = HardMix{make_double2(-1.0, 0.0), make_double2(0.0, -c.eta)};
                c.rn = make_double2(0.0, -c.eta);
                c.rd = make_double2(1.0, 0.0);
            }
    }
    return c;
}

// One H^2 matrix: tree, near field, couplings (everything but the composite case)
static igb_status build_one(igb_ctx ctx, igb_geom g, const igb_op_params* prm, const Coefs& c, igb_op* out) {
    igb_op op = new (std::nothrow) igb_op_s();
    if (!op) {
        set_error("assemble_nearfield: out of host memory");
        return IGB_ERR_ARG;
    }
    op->geom = g;
    op->prm = *prm;
    op->kappa = prm->kappa;
    op->bc = c.family;
    op->eta = c.eta;
    op->mix = c.mix;
    op->hmix = c.hmix;
    op->cm = c.cm;
    op->rn = c.rn;
    op->rd = c.rd;
    op->system = c.system;
    op->q = prm->q;
    op->nq = (prm->q + 1) * (prm->q + 1);
    op->N = op->bc == IGB_SOFT ? g->n2 : g->n0;
    igb_status st;
    if ((st = tree_build(op)) || (st = near_classify(op)) || (st = near_pattern(op))) {
        delete op;
        return st;
    }
    // device bytes of the operator (checked against the budget before allocating)
    const int nl = (g->p + 1) * (g->p + 1);
    const int ntile = op->bc == IGB_HARD ? 2 : 1;
    const size_t fp64_tiles =
        prm->far_on_the_fly ? 0 : size_t(op->nfar) * op->nq * op->nq * 16 * ntile + size_t(3) * op->nq * 16 + 256;
    size_t need = fp64_tiles + size_t(op->nnz) * 20 + size_t(op->N + 1) * 8 + op->near_dcol.size() * 4 +
                  op->row_coff.size() * 8 + op->near_wgs.size() * sizeof(NearGroupWG) +
                  op->near_grp_rows.size() * 4 +
                  size_t(op->nclusters) * op->nq * (16 * 8 + 32) + op->near_src.size() * 4;
    // held during assembly only: the staged element blocks and the near pair lists
    const size_t transient = std::min<size_t>(op->near_src.size(), size_t(1) << 22) * nl * nl * 16 +
                             op->near_src.size() * 12 + (size_t(1) << 20);
    // the near field in tiles: fp32 values (bf16 operators), fp64 values (fp64 and fp32 operators)
    if (op->nnz > 0)
        need += size_t(op->near_tile_vals) * (prm->precision == IGB_MIX_BF16 ? 8 : 16) +
                op->near_tiles.size() * sizeof(NearTile) + op->near_tile_cols.size() * 4;
    if (prm->precision != IGB_FP64) {
        // rounded tiles (rows padded to 16 bytes)
        const size_t esz = prm->precision == IGB_MIX_FP32 ? 8 : 4, epl = 16 / esz;
        const size_t ldk = (op->nq + epl - 1) / epl * epl;
        need += size_t(op->nfar) * ntile * op->nq * ldk * esz + size_t(3) * op->nq * 16 + 256;
    }
    // recompressed couplings: at most the tiles' size at the tolerances of interest
    if (prm->far_recompress_tol > 0) need += size_t(op->nfar) * op->nq * op->nq * 16 + size_t(op->nfar) * 12;
    op->estimated_data = need;
    // plus the matvec work vectors of one column and a GMRES(30) solve of one column
    // (more columns: igb_op_solve_bytes)
    need += work_sizes(op, 1).total() + solve_buffer_bytes(op, 30, 1) + quad_buffer_bytes(op, 1, 64);
    op->estimated_bytes = need;
    if (!budget_ok(ctx, need + transient)) {
        set_error("assemble_nearfield: HBM budget exceeded (%zu + %zu > %zu bytes)", ctx->used.load(),
                  need + transient, ctx->budget);
        delete op;
        return IGB_ERR_BUDGET;
    }
    hipStream_t s = ctx->stream;
    if (host_only(ctx)) {
        ++g->refs;
        *out = op;
        return IGB_OK;
    }
    if ((st = assemble_near_device(op, s)) || (st = assemble_far_device(op, s)) || (st = alloc_work(op, 1))) {
        delete op;
        return st;
    }
    ++g->refs;
    *out = op;
    return IGB_OK;
}


igb_status assemble_nearfield(igb_ctx ctx, igb_geom g, const igb_op_params* prm, igb_op* out) {
    if (!ctx || !g || !prm || !out) {
        set_error("assemble_nearfield: NULL argument");
        return IGB_ERR_ARG;
    }
    if (!(prm->kappa > 0) || prm->q < 1 || prm->q > QMAX || !(prm->eta_adm > 0) || prm->leaf_depth < 0 ||
        prm->leaf_depth > 6 ||
        (prm->bc != IGB_SOFT && prm->bc != IGB_HARD)) {
        set_error("assemble_nearfield: need kappa > 0, 1 <= q <= %d, eta_adm > 0, 0 <= leaf_depth <= 6, bc soft/hard",
                  QMAX);
        return IGB_ERR_ARG;
    }
    if (prm->precision != IGB_FP64 && prm->precision != IGB_MIX_FP32 && prm->precision != IGB_MIX_BF16) {
        set_error("assemble_nearfield: precision must be IGB_FP64, IGB_MIX_FP32 or IGB_MIX_BF16");
        return IGB_ERR_ARG;
    }
    if (prm->far_on_the_fly != 0 && prm->far_on_the_fly != 1) {
        set_error("assemble_nearfield: far_on_the_fly must be 0 or 1");
        return IGB_ERR_ARG;
    }
    if (prm->quad_extra < -2 || prm->quad_extra > 3) {
        set_error("assemble_nearfield: need -2 <= quad_extra <= 3");
        return IGB_ERR_ARG;
    }
    if (prm->formulation < IGB_CFIE || prm->formulation > IGB_OP_W) {
        set_error("assemble_nearfield: formulation must be IGB_CFIE, IGB_SINGLE_LAYER or IGB_OP_V / _KSTAR / _K / _W");
        return IGB_ERR_ARG;
    }
    if (prm->separate != 0 && (prm->separate != 1 || prm->formulation != IGB_CFIE)) {
        set_error("assemble_nearfield: separate must be 0, or 1 with IGB_CFIE");
        return IGB_ERR_ARG;
    }
    if (!(prm->far_recompress_tol >= 0 && prm->far_recompress_tol <= 1e-2)) {
        set_error("assemble_nearfield: need 0 <= far_recompress_tol <= 1e-2");
        return IGB_ERR_ARG;
    }
    const Coefs c = coefs_for(prm);
    if (prm->far_recompress_tol > 0 && (c.family != IGB_SOFT || prm->far_on_the_fly || prm->q > 7)) {
        set_error("assemble_nearfield: far_recompress_tol needs a sound-soft-family operator with stored couplings "
                  "and q <= 7");
        return IGB_ERR_UNSUPPORTED;
    }
    if (c.family == IGB_HARD && g->p < 1) {
        set_error("assemble_nearfield: the sound-hard operators need S^0, i.e. p >= 1");
        return IGB_ERR_ARG;
    }
    AllocScope scope(ctx);
    if (!host_only(ctx)) IGB_HIP(hipSetDevice(ctx->device));
    if (!prm->separate) return build_one(ctx, g, prm, c, out);

    // One H^2 matrix per operator of the CFIE (soft: 1/2 M + K* and V; hard: 1/2 M - K
    // and W), applied as the lazy sum part_0 + coef_1 part_1 (coef_1 = -i eta)
    Coefs c0 = c, c1 = c;
    c0.system = c1.system = false;
    c1.cm = make_double2(0, 0);
    if (c.family == IGB_SOFT) {
        c0.mix = SoftMix{1.0, make_double2(0, 0)};
        c1.mix = SoftMix{0.0, make_double2(1.0, 0)};
    } else {
        c0.hmix = HardMix{make_double2(-1.0, 0), make_double2(0, 0)};
        c1.hmix = HardMix{make_double2(0, 0), make_double2(1.0, 0)};
    }
    igb_op p0 = nullptr, p1 = nullptr;
    igb_status st;
    if ((st = build_one(ctx, g, prm, c0, &p0))) return st;
    if ((st = build_one(ctx, g, prm, c1, &p1))) {
        igb_op_destroy(p0);
        return st;
    }
    igb_op op = new (std::nothrow) igb_op_s();
    if (!op) {
        igb_op_destroy(p0);
        igb_op_destroy(p1);
        set_error("assemble_nearfield: out of host memory");
        return IGB_ERR_ARG;
    }
    op->geom = g;
    op->prm = *prm;
    op->kappa = prm->kappa;
    op->bc = c.family;
    op->eta = c.eta;
    op->mix = c.mix;
    op->hmix = c.hmix;
    op->cm = c.cm;
    op->rn = c.rn;
    op->rd = c.rd;
    op->system = true;
    op->q = p0->q;
    op->nq = p0->nq;
    op->N = p0->N;
    op->kd_elem = p0->kd_elem;
    op->aspect_max = p0->aspect_max;
    op->sum_parts = {p0, p1};
    op->sum_coef = {make_double2(1.0, 0.0), make_double2(0.0, -c.eta)};
    op->estimated_data = p0->estimated_data + p1->estimated_data;
    op->estimated_bytes = solve_model_bytes(op, 30, 1);
    ++g->refs;
    *out = op;
    return IGB_OK;
}

void igb_op_destroy(igb_op op) {
    if (!op) return;
    igb_geom g = op->geom;
    igb_ctx ctx = g->ctx;
    if (!host_only(ctx)) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
    }
    for (igb_op part : op->sum_parts) igb_op_destroy(part);
    op->sum_parts.clear();
    delete op;
    geom_release(g);
}

igb_status igb_op_get_info(igb_op op, igb_op_info* info) {
    if (!op || !info) {
        set_error("igb_op_get_info: NULL argument");
        return IGB_ERR_ARG;
    }
    std::memset(info, 0, sizeof(*info));
    if (!op->sum_parts.empty()) {
        // separate H^2 matrices: the tree of the first, sizes and times summed over all
        igb_op_get_info(op->sum_parts.front(), info);
        info->n = op->N;
        info->far_pairs = info->near_elem_pairs = info->nnz = 0;
        info->device_bytes = int64_t(op->dev_bytes);
        info->estimated_bytes = int64_t(op->estimated_bytes);
        info->assembly_near_ms = info->assembly_far_ms = 0;
        for (igb_op part : op->sum_parts) {
            igb_op_info pi;
            igb_op_get_info(part, &pi);
            info->far_pairs += pi.far_pairs;
            info->near_elem_pairs += pi.near_elem_pairs;
            info->nnz += pi.nnz;
            info->device_bytes += pi.device_bytes;
            info->assembly_near_ms += pi.assembly_near_ms;
            info->assembly_far_ms += pi.assembly_far_ms;
        }
        return IGB_OK;
    }
    info->n = op->N;
    info->nelem = op->geom->nelem;
    info->n2 = op->geom->n2;
    info->nclusters = op->nclusters;
    info->leaf_level = op->L;
    info->nq = op->nq;
    info->far_pairs = op->nfar;
    for (int l = 0; l <= op->L && l < 16; ++l) info->far_per_level[l] = int64_t(op->far[l].src.size());
    info->near_elem_pairs = int64_t(op->near_src.size());
    info->nnz = op->nnz;
    info->device_bytes = int64_t(op->dev_bytes);
    info->estimated_bytes = int64_t(op->estimated_bytes);
    info->assembly_near_ms = op->t_assembly_near;
    info->assembly_far_ms = op->t_assembly_far;
    info->far_factor_entries = op->lr_entries;
    info->near_col_entries = int64_t(op->near_dcol.size());
    info->near_tile_entries = int64_t(op->near_tile_vals);
    info->near_group_staged = !op->near_wgs.empty() &&
                              size_t(op->near_list_max) * 16 <= size_t(op->geom->ctx->lds_max) ? 1 : 0;
    return IGB_OK;
}

int64_t igb_op_ndof(igb_op op) { return op ? op->N : -1; }

int64_t igb_op_bytes(igb_op op) { return op ? int64_t(op_held_bytes(op)) : -1; }

igb_status igb_op_solve_bytes(igb_op op, int ndir, int restart, int64_t* bytes) {
    if (!op || !bytes || ndir < 1 || restart < 0) {
        set_error("igb_op_solve_bytes: invalid argument");
        return IGB_ERR_ARG;
    }
    *bytes = int64_t(solve_model_bytes(op, restart > 0 ? restart : 30, ndir));
    return IGB_OK;
}

igb_status igb_op_near_csr(igb_op op, int64_t* row_ptr, int32_t* col, double* val) {
    if (!op || !row_ptr || !col || !val) {
        set_error("igb_op_near_csr: NULL argument");
        return IGB_ERR_ARG;
    }
    if (igb_status st0 = need_single_matrix(op, "igb_op_near_csr")) return st0;
    igb_status st = need_device(op, "igb_op_near_csr");
    if (st) return st;
    IGB_HIP(hipSetDevice(op->geom->ctx->device));
    std::memcpy(row_ptr, op->row_ptr.data(), op->row_ptr.size() * sizeof(int64_t));
    std::memcpy(col, op->col.data(), op->col.size() * sizeof(int32_t));
    IGB_HIP(hipMemcpy(val, op->d_val.ptr, op->nnz * sizeof(double2), hipMemcpyDeviceToHost));
    return IGB_OK;
}

igb_status igb_op_far_blocks(igb_op op, int32_t* out) {
    if (!op || !out) {
        set_error("igb_op_far_blocks: NULL argument");
        return IGB_ERR_ARG;
    }
    if (igb_status st0 = need_single_matrix(op, "igb_op_far_blocks")) return st0;
    int64_t i = 0;
    for (int l = 0; l <= op->L; ++l) {
        const FarLevel& F = op->far[l];
        const int64_t nc = clusters_on_level(op->geom->npatch, l);
        for (int64_t t = 0; t < nc; ++t)
            for (int k = F.tgt_ptr[t]; k < F.tgt_ptr[t + 1]; ++k) {
                out[4 * i] = l;
                out[4 * i + 1] = int32_t(t);
                out[4 * i + 2] = F.src[k];
                out[4 * i + 3] = 0;
                ++i;
            }
    }
    return IGB_OK;
}

igb_status igb_op_potential_plan(igb_op op, const double* points, int npts, int64_t* counts, int32_t* perm,
                                 int32_t* box_ptr) {
    if (!op || !points || !counts || npts < 1) {
        set_error("igb_op_potential_plan: invalid argument");
        return IGB_ERR_ARG;
    }
    for (int64_t i = 0; i < 3 * int64_t(npts); ++i)
        if (!std::isfinite(points[i])) {
            set_error("igb_op_potential_plan: point %lld is not finite", (long long)(i / 3));
            return IGB_ERR_ARG;
        }
    // the geometry and q of the first part of a separate-form operator, as potential_h2
    const igb_op sp = op->sum_parts.empty() ? op : op->sum_parts.front();
    PotentialPlan P;
    if (igb_status st = potential_plan(sp, points, npts, P)) return st;
    counts[0] = int64_t(P.box_ptr.size()) - 1;
    counts[1] = int64_t(P.far_src.size());
    counts[2] = int64_t(P.m2p_src.size());
    counts[3] = int64_t(P.near_leaf.size());
    if (perm) std::memcpy(perm, P.perm.data(), P.perm.size() * sizeof(int32_t));
    if (box_ptr) std::memcpy(box_ptr, P.box_ptr.data(), P.box_ptr.size() * sizeof(int32_t));
    return IGB_OK;
}

igb_status igb_op_near_pairs(igb_op op, int64_t* ptr, int32_t* src, int32_t* kind) {
    if (!op || !ptr || !src || !kind) {
        set_error("igb_op_near_pairs: NULL argument");
        return IGB_ERR_ARG;
    }
    if (igb_status st0 = need_single_matrix(op, "igb_op_near_pairs")) return st0;
    std::memcpy(ptr, op->near_ptr.data(), op->near_ptr.size() * sizeof(int64_t));
    std::memcpy(src, op->near_src.data(), op->near_src.size() * sizeof(int32_t));
    std::memcpy(kind, op->near_kind.data(), op->near_kind.size() * sizeof(int32_t));
    return IGB_OK;
}

igb_status igb_geom_s0_map(igb_geom g, int32_t* s2_to_s0) {
    if (!g || !s2_to_s0) {
        set_error("igb_geom_s0_map: NULL argument");
        return IGB_ERR_ARG;
    }
    std::memcpy(s2_to_s0, g->s2_to_s0.data(), g->s2_to_s0.size() * sizeof(int32_t));
    return IGB_OK;
}

igb_status igb_op_profile(igb_op op, int enable) {
    if (!op) {
        set_error("igb_op_profile: NULL argument");
        return IGB_ERR_ARG;
    }
    if (igb_status st0 = need_single_matrix(op, "igb_op_profile")) return st0;
    op->profile = enable != 0;
    for (auto& t : op->timers) t.used = 0;
    return IGB_OK;
}

igb_status igb_op_use_graphs(igb_op op, int enable) {
    if (!op) {
        set_error("igb_op_use_graphs: NULL argument");
        return IGB_ERR_ARG;
    }
    op->use_graphs = enable != 0;
    if (!op->use_graphs) op->clear_graphs();
    for (igb_op part : op->sum_parts) igb_op_use_graphs(part, enable);
    return IGB_OK;
}

igb_status igb_op_set_tile_shape(igb_op op, int coupling_col_tiles, int near_col_tiles) {
    if (!op) {
        set_error("igb_op_set_tile_shape: NULL argument");
        return IGB_ERR_ARG;
    }
    auto ok = [](int v) { return v == 0 || v == 1 || v == 2 || v == 4; };
    if (!ok(coupling_col_tiles) || !ok(near_col_tiles)) {
        set_error("igb_op_set_tile_shape: column tiles must be 0, 1, 2 or 4 (got %d, %d)", coupling_col_tiles,
                  near_col_tiles);
        return IGB_ERR_ARG;
    }
    op->tile_m2l_nc = coupling_col_tiles;
    op->tile_near_nct = near_col_tiles;
    op->clear_graphs();
    for (igb_op part : op->sum_parts) igb_op_set_tile_shape(part, coupling_col_tiles, near_col_tiles);
    return IGB_OK;
}

igb_status igb_op_kernel_time(igb_op op, const char* name, int64_t* launches, double* total_ms) {
    if (!op || !name || !launches || !total_ms) {
        set_error("igb_op_kernel_time: NULL argument");
        return IGB_ERR_ARG;
    }
    if (igb_status st0 = need_single_matrix(op, "igb_op_kernel_time")) return st0;
    static const char* names[4] = {"m2l", "spmv", "upward", "downward"};
    int slot = -1;
    for (int i = 0; i < 4; ++i)
        if (std::strcmp(name, names[i]) == 0) slot = i;
    if (slot < 0) {
        set_error("igb_op_kernel_time: unknown kernel '%s' (m2l, spmv, upward, downward)", name);
        return IGB_ERR_ARG;
    }
    KernelTimer& t = op->timers[slot];
    double tot = 0;
    for (size_t i = 0; i + 1 < t.used; i += 2) {
        IGB_HIP(hipEventSynchronize(t.pool[i + 1]));
        float ms = 0;
        IGB_HIP(hipEventElapsedTime(&ms, t.pool[i], t.pool[i + 1]));
        tot += ms;
    }
    *launches = int64_t(t.used / 2);
    *total_ms = tot;
    t.used = 0;
    return IGB_OK;
}

igb_status h2_matvec(igb_op op, const double* x, double* y, int nrhs, int parts, void* hip_stream) {
    if (!op || !x || !y || nrhs < 1 || (parts & 3) == 0 || parts > 15) {
        set_error("h2_matvec: invalid argument");
        return IGB_ERR_ARG;
    }
    if (x == y) {
        set_error("h2_matvec: x and y must not overlap");
        return IGB_ERR_ARG;
    }
    if (igb_status st = need_device(op, "h2_matvec")) return st;
    AllocScope scope(op->geom->ctx);
    IGB_HIP(hipSetDevice(op->geom->ctx->device));
    hipStream_t s = pick(op->geom->ctx, hip_stream);
    if (!(parts & IGB_MV_HOST)) return matvec_device(op, x, y, nrhs, parts, s);
    // host columns: stage through operator-owned device buffers
    const size_t bytes = size_t(nrhs) * op->N * 16;
    igb_status st;
    if ((st = op_reserve(op, op->d_hx, bytes, "h2_matvec")) || (st = op_reserve(op, op->d_hy, bytes, "h2_matvec")))
        return st;
    IGB_HIP(hipMemcpyAsync(op->d_hx.ptr, x, bytes, hipMemcpyHostToDevice, s));
    if ((st = matvec_device(op, op->d_hx.as<double>(), op->d_hy.as<double>(), nrhs, parts & ~IGB_MV_HOST, s)))
        return st;
    IGB_HIP(hipMemcpyAsync(y, op->d_hy.ptr, bytes, hipMemcpyDeviceToHost, s));
    IGB_HIP(hipStreamSynchronize(s));
    return IGB_OK;
}

igb_status h2_matvec_noalloc(igb_op op, const double* x, double* y, int nrhs, int parts, void* hip_stream) {
    if (!op || !x || !y || nrhs < 1 || (parts & 3) == 0 || parts > 7) {
        set_error("h2_matvec_noalloc: invalid argument (device arrays only; IGB_MV_HOST is not accepted)");
        return IGB_ERR_ARG;
    }
    if (x == y) {
        set_error("h2_matvec_noalloc: x and y must not overlap");
        return IGB_ERR_ARG;
    }
    if (igb_status st = need_device(op, "h2_matvec_noalloc")) return st;
    if (!op->sum_parts.empty()) {
        set_error("h2_matvec_noalloc: not available on an operator stored as separate H^2 matrices");
        return IGB_ERR_UNSUPPORTED;
    }
    if (op->profile) {
        set_error("h2_matvec_noalloc: per-kernel profiling is enabled on the operator (it records events)");
        return IGB_ERR_ARG;
    }
    IGB_HIP(hipSetDevice(op->geom->ctx->device));
    return matvec_noalloc(op, x, y, nrhs, parts, pick(op->geom->ctx, hip_stream));
}

igb_status cfie_rhs(igb_op op, const double* dirs, int ndir, double* b, void* hip_stream) {
    if (!op || !dirs || !b || ndir < 1) {
        set_error("cfie_rhs: invalid argument");
        return IGB_ERR_ARG;
    }
    if (igb_status st = need_device(op, "cfie_rhs")) return st;
    AllocScope scope(op->geom->ctx);
    if (igb_status st1 = need_system(op, "cfie_rhs")) return st1;
    IGB_HIP(hipSetDevice(op->geom->ctx->device));
    return rhs_device(op, dirs, ndir, b, pick(op->geom->ctx, hip_stream));
}

igb_status cfie_solve(igb_op op, const double* dirs, int ndir, const igb_solve_params* sp, double* coeffs,
                      igb_solve_info* info) {
    if (!op || !dirs || !sp || !coeffs || ndir < 1) {
        set_error("cfie_solve: invalid argument");
        return IGB_ERR_ARG;
    }
    if (igb_status st1 = need_system(op, "cfie_solve")) return st1;
    {
        // the solve's growth, from the size model, against the budget before any work
        igb_ctx ctx = op->geom->ctx;
        const size_t model = solve_model_bytes(op, sp->restart > 0 ? sp->restart : 30, ndir);
        const size_t held = host_only(ctx) ? 0 : op_held_bytes(op);
        const size_t grow = model > held ? model - held : 0;
        if (!budget_ok(ctx, grow)) {
            set_error("cfie_solve: HBM budget exceeded by %d directions (%zu held + %zu > %zu bytes)", ndir,
                      ctx->used.load(), grow, ctx->budget);
            return IGB_ERR_BUDGET;
        }
    }
    if (igb_status st0 = need_device(op, "cfie_solve")) return st0;
    AllocScope scope(op->geom->ctx);
    IGB_HIP(hipSetDevice(op->geom->ctx->device));
    hipStream_t s = op->geom->ctx->stream;
    const auto t_start = std::chrono::steady_clock::now();
    // right-hand sides in an operator-owned buffer (kept for later solves)
    igb_status st = op_reserve(op, op->d_b, size_t(ndir) * op->N * 16, "cfie_solve");
    if (st) return st;
    if ((st = rhs_device(op, dirs, ndir, op->d_b.as<double>(), s))) return st;
    st = gmres_device(op, op->d_b.as<double>(), coeffs, ndir, sp, info, s);
    IGB_HIP(hipStreamSynchronize(s));
    if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return st;
}

igb_status farfield(igb_op op, const double* coeffs, int ndir, const double* obs, int nobs, double* uinf,
                    void* hip_stream) {
    if (!op || !coeffs || !obs || !uinf || ndir < 1 || nobs < 1) {
        set_error("farfield: invalid argument");
        return IGB_ERR_ARG;
    }
    if (igb_status st = need_device(op, "farfield")) return st;
    AllocScope scope(op->geom->ctx);
    if (igb_status st1 = need_system(op, "farfield")) return st1;
    IGB_HIP(hipSetDevice(op->geom->ctx->device));
    return farfield_device(op, coeffs, ndir, obs, nobs, uinf, pick(op->geom->ctx, hip_stream));
}

igb_status potential(igb_op op, const double* coeffs, int ndir, const double* points, int npts, double* u,
                     void* hip_stream) {
    if (!op || !coeffs || !points || !u || ndir < 1 || npts < 1) {
        set_error("potential: invalid argument");
        return IGB_ERR_ARG;
    }
    if (igb_status st = need_device(op, "potential")) return st;
    AllocScope scope(op->geom->ctx);
    if (igb_status st1 = need_system(op, "potential")) return st1;
    IGB_HIP(hipSetDevice(op->geom->ctx->device));
    return potential_device(op, coeffs, ndir, points, npts, u, pick(op->geom->ctx, hip_stream));
}

igb_status potential_h2(igb_op op, const double* coeffs, int ndir, const double* points, int npts, double* u,
                     void* hip_stream) {
    if (!op || !coeffs || !points || !u || ndir < 1 || npts < 1) {
        set_error("potential_h2: invalid argument");
        return IGB_ERR_ARG;
    }
    if (igb_status st = need_device(op, "potential_h2")) return st;
    AllocScope scope(op->geom->ctx);
    if (igb_status st1 = need_system(op, "potential_h2")) return st1;
    IGB_HIP(hipSetDevice(op->geom->ctx->device));
    return potential_h2_device(op, coeffs, ndir, points, npts, u, pick(op->geom->ctx, hip_stream));
}

}  // extern "C"

// Internal definitions of the igafmm library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <mutex>
#include <new>
#include <utility>
#include <cstdint>
#include <cstdio>
#include <string>
#include <thread>
#include <vector>

#include "../../include/igafmm.h"

namespace igb {

constexpr int PMAX = 3;         // spline degree of the discrete spaces
constexpr int PGMAX = 3;        // polynomial degree of the geometry per element
constexpr int NBZ = (PGMAX + 1) * (PGMAX + 1);
constexpr int QMAX = 10;        // interpolation degree
constexpr int NLOCMAX = (PMAX + 1) * (PMAX + 1);

// Kernel of the sound-soft family of operators: ck K* + cv V (complex cv)
struct SoftMix {
    double ck;
    double2 cv;
};

// Kernel of the sound-hard family: ck K + cw W (complex ck, cw)
struct HardMix {
    double2 ck;
    double2 cw;
};

// thread-local error message set by every failing entry point
void set_error(const char* fmt, ...);

#define IGB_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::igb::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call,           \
                             hipGetErrorString(e_));                               \
            return IGB_ERR_HIP;                                                    \
        }                                                                          \
    } while (0)

}  // namespace igb

struct igb_ctx_s {
    int refs = 1;        // the caller's handle + one per live geometry
    int device = 0;
    size_t budget = 0;   // bytes the library may hold on this device (0 = no limit)
    // bytes currently held on the device: every allocation of the context's
    // geometries and operators (tables, work vectors, Krylov bases, temporaries)
    std::atomic<size_t> used{0};
    hipStream_t stream = nullptr;
    int lds_max = 0;     // LDS bytes a workgroup may allocate
};

namespace igb {

// HBM budget accounting.  Every device allocation of the library is charged to
// a context: the one whose entry point runs on this thread (set by AllocScope
// at each entry point); the buffer remembers it and credits the bytes back
// when released.  charge() fails, changing nothing, if the budget would be
// exceeded.
igb_ctx_s*& alloc_ctx();
struct AllocScope {
    igb_ctx_s* prev;
    explicit AllocScope(igb_ctx_s* c) : prev(alloc_ctx()) { alloc_ctx() = c; }
    ~AllocScope() { alloc_ctx() = prev; }
};
bool charge(igb_ctx_s* c, size_t bytes);
inline void uncharge(igb_ctx_s* c, size_t bytes) { c->used.fetch_sub(bytes); }

// ----------------------------------------------------------------------------
// device memory owned by a handle; freed in the destructor
// ----------------------------------------------------------------------------
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    igb_ctx_s* ctx = nullptr;   // context charged for the bytes
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (ptr) (void)hipFree(ptr);
        if (ctx) uncharge(ctx, bytes);
        ptr = nullptr;
        bytes = 0;
        ctx = nullptr;
    }
    template <class T> T* as() const { return static_cast<T*>(ptr); }
};

// Releases b, then allocates `bytes` charged to alloc_ctx(): IGB_ERR_BUDGET
// (message naming `who`) if that context's budget would be exceeded,
// IGB_ERR_HIP if hipMalloc fails; b is empty after either.
igb_status dev_malloc(DevBuf& b, size_t bytes, const char* who);
// As dev_malloc, but keeps b when it already holds at least `bytes`.
inline igb_status dev_reserve(DevBuf& b, size_t bytes, const char* who) {
    return b.bytes >= bytes && b.ptr ? IGB_OK : dev_malloc(b, bytes, who);
}

}  // namespace igb

// Per-element data of a discretised geometry.
struct igb_geom_s {
    int refs = 1;                // the caller's handle + one per live operator
    igb_ctx ctx = nullptr;
    int npatch = 0, m = 0, p = 0, nel1 = 0, k = 0;
    int64_t nelem = 0, n2 = 0, n0 = 0;
    // host copies
    std::vector<double> bez;     // [E][NBZ][4]: homogeneous rational Bezier net of the element
    std::vector<int> pg;         // [E][2]: geometry degree in u and v
    std::vector<double> lo, hi;  // [E][3]: box of the projected Bezier control points
    std::vector<int> espan;      // [E][2]: index of the geometry knot span (u, v) holding the element
    std::vector<double> corner;  // [E][4][3]: physical corners at local (0,0),(1,0),(0,1),(1,1)
    std::vector<int> vert;       // [E][4]: global vertex id of each corner
    std::vector<double> C1;      // [nel1][p+1][p+1]: b_{ex+a} = sum_k C1[ex][a][k] Bernstein_k
    std::vector<int> s2_to_s0;   // [n2]
    std::vector<int> s0_ptr;     // [n0+1]  S^0 dof -> its S^2 representatives
    std::vector<int> s0_reps;    // [n2]
    // device copies
    igb::DevBuf d_bez, d_pg, d_C1;
    size_t dev_bytes = 0;
};

// HIP-event timing of selected kernel launches (enabled per operator)
struct KernelTimer {
    std::vector<hipEvent_t> pool;   // pairs (start, stop)
    size_t used = 0;                // events recorded since the last query
};

struct FarLevel {
    int level = 0;
    int64_t pair_off = 0;        // first far pair of this level (global pair index)
    std::vector<int> tgt_ptr;    // CSR over target clusters of the level (npatch*4^l + 1)
    std::vector<int> src;        // source cluster (local index in the level) per pair
};

// M2L work decomposition: chunks of consecutive far pairs of one target; each
// chunk produces one partial result, summed per target in chunk order
constexpr int M2L_CHUNK = 8;
constexpr int M2L_CHUNK_MFMA = 16;
constexpr int64_t M2L_MFMA_CHUNKS_MIN = 1024;
struct M2LChunks {
    std::vector<int> tgt;       // global cluster index of the chunk's target
    std::vector<int64_t> pair;  // first pair of the chunk
    std::vector<int> len;
    std::vector<int> tgt_ptr;   // [nclusters+1] chunks per target (global index)
    igb::DevBuf d_tgt, d_pair, d_len, d_tgt_ptr;
};

// Near rows whose supports lie in the same leaves have the same column list.
// Up to 16 rows of such groups form a tile over the union of their column
// lists; its values are stored [k block][row][8] (zeros where a row lacks a
// column and past the list's end, padded to a multiple of 8), the A operand
// of the matrix-core near product.
constexpr int NEAR_TILE_ROWS = 16;
constexpr int NEAR_TILE_K = 8;
constexpr double NEAR_TILE_FILL = 0.35;   // union at most 35% longer than the longest member list
// rows per workgroup of the group-staged one-column near product (one wave each)
constexpr int NEAR_GROUP_ROWS = 16;
struct NearGroupWG {
    int64_t list_off;   // the group's column list in near_dcol
    int list_len;       // its length (every row of the group has this many entries)
    int row0, nrows;    // the workgroup's rows: near_grp_rows[row0 .. row0 + nrows)
    int pad;
};

struct NearTile {
    int64_t val_off;   // first complex entry of the tile in the tile layout
    int64_t col_off;   // first entry of the tile's column list (sorted)
    int ncols, nrows;
    int rows[NEAR_TILE_ROWS];
};
// blocks of at least this many columns take the matrix-core paths of fp64
// operators (coupling and near product)
constexpr int MF64_MIN_COLS = 16;

struct igb_op_s {
    igb_geom geom = nullptr;
    igb_op_params prm{};
    int bc = 0;                   // operator family: IGB_SOFT (S^2, V and K*) or IGB_HARD (S^0, K and W)
    double kappa = 0, eta = 0;
    // system (cm M + ck K* + cv V) t = <(rn d_n + rd) u_inc, psi> of the soft family, or
    // (cm M + ck K + cw W) g = <(rn d_n + rd) u_inc, psi> of the hard one (mix / hmix)
    igb::SoftMix mix{1.0, {0.0, 0.0}};
    igb::HardMix hmix{{-1.0, 0.0}, {0.0, 0.0}};
    double2 cm{0.5, 0.0}, rn{1.0, 0.0}, rd{0.0, 0.0};
    int q = 0, nq = 0, L = 0, d = 0;
    double kd_elem = 0;           // kappa * largest element box diagonal
    double aspect_max = 1;        // largest ratio of an element's extents along u and v
    int64_t N = 0;
    // cluster indexing: level l holds npatch * 4^l clusters starting at clu_off[l]
    std::vector<int64_t> clu_off;
    std::vector<double> clo, chi;     // [nclusters][3] boxes
    std::vector<FarLevel> far;        // one entry per level 0..L
    int64_t nfar = 0;
    int far_lmin = 0;                 // coarsest level with admissible pairs (L + 1: none); moments and
                                      // expansions of coarser levels are neither formed nor transferred
    // near field: per target element the sorted near source elements
    std::vector<int64_t> near_ptr;    // [E+1]
    std::vector<int> near_src;
    std::vector<std::vector<int>> near_leaf;  // per leaf (local index): sorted inadmissible leaves
    std::vector<int> near_kind;       // per near pair: 0 regular (order in bits 8..), 1 vertex,
                                      // 2 edge, 4 identical; transforms in bits 16.. / 20..
    // near CSR in the solution space
    std::vector<int64_t> row_ptr;
    std::vector<int> col;
    int64_t nnz = 0;
    // rows with the same leaves have the same columns: each such list once (near_dcol)
    // and per row the offset of its list (the near products read columns from here)
    std::vector<int> near_dcol;
    std::vector<int64_t> row_coff;
    // the one-column near product by groups: workgroups of up to
    // NEAR_GROUP_ROWS rows of one group (rows listed group by group in
    // near_grp_rows), each staging its group's x entries in LDS once
    std::vector<NearGroupWG> near_wgs;
    std::vector<int> near_grp_rows;
    int near_list_max = 0;   // longest group column list
    // bf16 operators: the near rows in tiles of up to 16 rows over a common column list
    std::vector<NearTile> near_tiles;
    std::vector<int> near_tile_cols;  // the tiles' column lists
    int64_t near_tile_vals = 0;       // complex entries of the tile layout
    // M2L work decompositions (vector path, matrix-core path)
    M2LChunks chunks, chunks_mfma;
    // device data
    igb::DevBuf d_coupling, d_coupling_lo, d_nodes, d_m1, d_T, d_Tc;
    // recompressed couplings (far_recompress_tol > 0): per far pair the rank, the offset of
    // its factors (complex entries) and the factors u_k [k][nq], v_k^T [nq][rank]
    igb::DevBuf d_lr, d_lr_rank, d_lr_off;
    int64_t lr_entries = 0;
    igb::DevBuf d_rowptr, d_col, d_val, d_dcol, d_row_coff, d_near_wgs, d_near_grp_rows;
    // bf16 operators: fp32 near-field values and fp32 copies of the columns for the
    // near product of the inner (refinement) matvecs
    igb::DevBuf d_val_lo, d_xnear_lo, d_near_tiles, d_near_tile_cols;
    // fp64 operators: fp64 near-field values in the same tiles, for the near
    // product of blocks of >= 16 columns on the fp64 matrix cores
    igb::DevBuf d_val64;
    igb::DevBuf d_near_ptr, d_near_src;
    igb::DevBuf d_s2_to_s0, d_s0_ptr, d_s0_reps;
    igb::DevBuf d_far_src;
    // reduced-precision path: source vectors rounded per matvec, fp32 partials
    igb::DevBuf d_xlo, d_part_lo;
    igb::DevBuf d_xhat, d_yhat, d_yraw, d_part, d_x2, d_cluoff, d_leafbuf, d_xnear64;
    size_t dev_bytes = 0;
    int64_t nclusters = 0;
    // solver scratch (kept between solves, grown on demand): Krylov basis and
    // work vectors, Hessenberg steps, right-hand sides, refinement residual and
    // corrections
    igb::DevBuf d_krylov, d_w, d_h, d_b, d_dotpart, d_ref_r, d_ref_d, d_ref_d2;
    // device copies of host columns (h2_matvec with IGB_MV_HOST)
    igb::DevBuf d_hx, d_hy;
    // right-hand side and far-field buffers (kept between calls): Gauss table,
    // directions, element contributions, observation directions, quadrature
    // points and densities
    igb::DevBuf d_gauss, d_q_dirs, d_q_loc, d_q_obs, d_q_geo, d_q_dens;
    // false for a single boundary integral operator (no right-hand side or representation)
    bool system = true;
    // lazy sum y = sum_i sum_coef[i] sum_parts[i] x of separately stored H^2 matrices
    // (owned; empty for an operator with its own near and far field)
    std::vector<igb_op_s*> sum_parts;
    std::vector<double2> sum_coef;
    igb::DevBuf d_sum_tmp;
    int krylov_cols = 0;
    int work_cols = 0;   // columns the matvec work buffers are sized for
    double t_assembly_near = 0, t_assembly_far = 0;
    size_t estimated_bytes = 0;   // data + one-column work vectors + a GMRES(30) basis for one column
    size_t estimated_data = 0;    // operator data alone (tables, near field, couplings)
    // per-kernel timing: 0 m2l, 1 spmv, 2 upward, 3 downward
    bool profile = false;
    KernelTimer timers[4];
    // matvec launch sequences captured as HIP graphs, keyed by
    // (x, y, columns, parts, stream); cleared when the work buffers change
    struct GraphKey {
        const void* x;
        void* y;
        int ncol, parts;
        hipStream_t s;
        bool operator==(const GraphKey& o) const {
            return x == o.x && y == o.y && ncol == o.ncol && parts == o.parts && s == o.s;
        }
    };
    std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
    bool use_graphs = false;
    // tile shapes of the fp64 block kernels (0: automatic)
    int tile_m2l_nc = 0, tile_near_nct = 0;
    void clear_graphs() {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
        graphs.clear();
    }
    void* h_pin = nullptr;            // pinned host buffers of the GMRES Hessenberg steps (two)
    size_t h_pin_bytes = 0;
    hipEvent_t ev_h[2] = {nullptr, nullptr};   // their copies have landed
    ~igb_op_s() {
        if (h_pin) (void)hipHostFree(h_pin);
        for (hipEvent_t e : ev_h)
            if (e) (void)hipEventDestroy(e);
        clear_graphs();
        for (auto& t : timers)
            for (hipEvent_t e : t.pool) (void)hipEventDestroy(e);
    }
};

namespace igb {

// dev_reserve for a buffer owned by the operator, keeping its byte count
inline igb_status op_reserve(igb_op op, DevBuf& b, size_t bytes, const char* who) {
    if (b.bytes >= bytes && b.ptr) return IGB_OK;
    op->dev_bytes -= std::min(op->dev_bytes, b.bytes);
    const igb_status st = dev_malloc(b, bytes, who);
    op->dev_bytes += b.bytes;
    return st;
}

// host stages
igb_status geometry_build(igb_ctx ctx, const igb_patch* patches, int npatch, int m, int p,
                          igb_geom g);
igb_status tree_build(igb_op op);
igb_status near_classify(igb_op op);
igb_status near_pattern(igb_op op);

// device stages (kernels.hip)
igb_status upload_geometry(igb_geom g);
igb_status assemble_near_device(igb_op op, hipStream_t s);
igb_status assemble_far_device(igb_op op, hipStream_t s);
igb_status alloc_work(igb_op op, int nrhs);
// bytes of the matvec work buffers for ncol columns (alloc_work's sizes)
struct WorkSizes {
    enum { XHAT, YHAT, YRAW, PART, XLO, PART_LO, XNEAR_LO, X2, LEAFBUF, XNEAR64, COUNT };
    size_t b[COUNT];
    size_t total() const {
        size_t t = 0;
        for (size_t v : b) t += v;
        return t;
    }
};
WorkSizes work_sizes(const igb_op_s* op, int ncol);
// device addresses of the matvec work buffers (the operator's own, or carved out
// of the per-device scratch array by the allocation-free matvec)
struct MatvecWork {
    double2 *xhat = nullptr, *yhat = nullptr, *yraw = nullptr, *part = nullptr;
    void *xlo = nullptr, *part_lo = nullptr;
    float2* xnear_lo = nullptr;
    double2 *x2 = nullptr, *leafbuf = nullptr;
    double2* xnear64 = nullptr;   // transposed fp64 columns of the tile near product
};
constexpr int SCRATCH_MAX_DEVICES = 64;
// takes the device address of the scratch array of the current device (once per device)
igb_status scratch_init(int device);
// y = A x with the work buffers in the scratch array; allocates nothing
igb_status matvec_noalloc(igb_op op, const double* x, double* y, int ncol, int parts, hipStream_t s);
igb_status matvec_device(igb_op op, const double* x, double* y, int nrhs, int parts,
                         hipStream_t s);
igb_status rhs_device(igb_op op, const double* dirs, int ndir, double* b, hipStream_t s);
igb_status farfield_device(igb_op op, const double* coeffs, int ndir, const double* obs,
                           int nobs, double* uinf, hipStream_t s);
igb_status potential_device(igb_op op, const double* coeffs, int ndir, const double* points, int npt, double* u,
                            hipStream_t s);
// Extra Gauss points per direction for a wavenumber-scaled size kd = kappa * diameter:
// one more for each doubling of kd beyond 1.5 (oscillation of e^{i kappa r} across it).
inline int kd_boost(double kd) { return (kd >= 1.5) + (kd >= 3.0) + (kd >= 6.0); }
constexpr int REG_POINTS_MAX = 100;  // Gauss points per element of a regular near pair
// Extra points per direction of the touching-pair rules for elements much longer
// in one direction than in the other (the rules see the singularity through the
// reference square, where such an element squeezes it along one axis).
inline int aspect_boost(double a) { return (a >= 2.0) + (a >= 3.0) + (a >= 5.0); }
// Gauss orders per direction and element of the surface integrals that carry
// no singularity: right-hand side and far field (base 6), potential off the
// boundary (base 8); raised with kappa * element size and quad_extra > 0.
int smooth_order(igb_op op, int base);
// H^2 evaluation of the scattered field at many points (host plan).  Sources:
// the patch quadtrees down to level lmax = max(m - 1, 0) (clusters of 4
// elements), independent of the operator's leaf depth.  Targets: the points
// sorted into the boxes of an octree (at most POT_LEAF_POINTS each).  Per box:
// the source clusters admissible for both sides (far, interpolated on (q+1)^3
// box nodes; taken only where the box holds more points than nodes), those
// admissible for the source side (m2p: their interpolation nodes act on the
// box's points directly) and the inadmissible clusters of level lmax (near,
// direct quadrature).
constexpr int POT_LEAF_POINTS = 128;
// allocator whose resize leaves ints uninitialised (for lists filled right after)
template <class T>
struct UninitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = UninitAlloc<U>;
    };
    UninitAlloc() = default;
    template <class U>
    UninitAlloc(const UninitAlloc<U>&) {}
    template <class U>
    void construct(U* p) noexcept {
        ::new (static_cast<void*>(p)) U;
    }
    template <class U, class... A>
    void construct(U* p, A&&... a) {
        ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
    }
};
using IdList = std::vector<int, UninitAlloc<int>>;

struct PotentialPlan {
    int lmax = 0;                          // finest source level
    std::vector<int64_t> off;              // [lmax+2] first global id of each source level
    std::vector<int> perm;                 // points by box: perm[i] = caller's index
    std::vector<int> box_ptr;              // [nbox+1] into perm
    std::vector<double> box_lo, box_hi;    // [nbox][3] interpolation boxes
    // per box (ptr into the flat list): global ids of the clusters interpolated on
    // the box, global ids of those evaluated at the points, and the clusters of
    // level lmax summed directly (index on the level)
    std::vector<int> far_ptr, m2p_ptr, near_ptr;
    IdList far_src, m2p_src, near_leaf;
};
igb_status potential_plan(igb_op op, const double* points, int npts, PotentialPlan& P);
igb_status potential_h2_device(igb_op op, const double* coeffs, int ndir, const double* points, int npt, double* u,
                               hipStream_t s);
igb_status gmres_device(igb_op op, const double* b, double* x, int ndir,
                        const igb_solve_params* sp, igb_solve_info* info, hipStream_t s);
// bytes of cfie_solve's own buffers for ndir columns and restart m: Krylov basis,
// work vectors, Hessenberg steps, inner-product partials, right-hand sides and
// (reduced-precision operators) the refinement residual and corrections
size_t solve_buffer_bytes(const igb_op_s* op, int m, int ndir);
// device bytes an operator holds after cfie_solve(ndir, restart m) and a far
// field of its ndir columns at nobs directions: its data, the matvec work
// vectors of ndir columns, solve_buffer_bytes and quad_buffer_bytes
size_t solve_model_bytes(const igb_op_s* op, int m, int ndir, int nobs = 64);
// bytes of the right-hand side and far-field buffers (Gauss table, directions,
// element contributions, quadrature points and densities)
size_t quad_buffer_bytes(const igb_op_s* op, int ndir, int nobs);

// kernel timing helpers (no-ops unless op->profile)
igb_status timer_mark(igb_op op, int slot, hipStream_t s);
// admissibility helpers
inline int64_t clusters_on_level(int npatch, int l) { return int64_t(npatch) << (2 * l); }

// Host threads for the plan stages: the CPUs this process may run on, at most 16.
int host_threads();

// f(i) for every i in [0, n), in blocks of `grain` handed out dynamically to
// host_threads() threads (the calling thread is one of them).
template <class F>
void parallel_for(int64_t n, int64_t grain, const F& f) {
    const int64_t blocks = (n + grain - 1) / grain;
    const int nt = int(std::min<int64_t>(host_threads(), blocks));
    if (nt <= 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int64_t> next{0};
    auto run = [&]() {
        for (;;) {
            const int64_t a = next.fetch_add(grain);
            if (a >= n) return;
            const int64_t b = std::min(n, a + grain);
            for (int64_t i = a; i < b; ++i) f(i);
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(run);
    run();
    for (auto& t : pool) t.join();
}

// Chebyshev points of the first kind on [0,1]
void cheb_nodes(int q, double* t);

}  // namespace igb

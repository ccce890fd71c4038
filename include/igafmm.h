/*
 * igafmm -- isogeometric fast-multipole Galerkin CFIE for acoustic scattering
 * (Doelz, Harbrecht, Multerer: "Solving acoustic scattering problems by the
 * isogeometric boundary element method").  C ABI of the MI355X (gfx950) library.
 *
 * General conventions
 *   - Every entry point returns an igb_status: 0 = success, < 0 = error (nothing
 *     written to outputs), > 0 = warning (outputs written).  The text of the
 *     last error of the calling thread is returned by igb_last_error().
 *   - Complex numbers are interleaved (re, im) fp64 pairs, compatible with
 *     C99 double _Complex and torch.complex128.  Multi-column arrays are
 *     column-major in the sense [ncol][n]: each column contiguous.
 *   - "host" pointers are read or written synchronously.  "device" pointers
 *     must point to device memory of the context's GPU; calls that take a
 *     hip_stream argument are ordered on that stream (NULL = the device's null
 *     stream, IGB_CONTEXT_STREAM = the context's own non-blocking stream) and
 *     return before the device work completes.
 *   - The caller owns every buffer it passes; the library copies what it keeps.
 *     Handles own their device memory until destroyed; they may be destroyed in
 *     any order (an operator keeps its geometry, a geometry its context alive
 *     until the last dependent handle is destroyed).  Calls on one operator
 *     (h2_matvec, cfie_rhs, cfie_solve, farfield, potential, potential_h2) use
 *     its internal work vectors and must not overlap; different operators may
 *     run concurrently on different streams.  Work buffers grow on demand and
 *     stay with the operator until it is destroyed, so repeated calls of the
 *     same size allocate nothing.
 *
 * Numbering (patch-major):
 *   elements  e = patch*4^m + ey*2^m + ex  covering [ex,ex+1]x[ey,ey+1]/2^m of the
 *             patch's reference square;
 *   S^2 dofs  i = patch*k^2 + iv*k + iu,  k = 2^m + p: the tensor B-spline
 *             b_iu(u) b_iv(v) of S_{p,p}(Xi_{p,m}, Xi_{p,m}) on the patch (Sec. 3.3);
 *   S^0 dofs  the globally continuous subspace (Sec. 3.3): an S^0 function is the
 *             sum of the S^2 functions whose Greville anchor points coincide on
 *             patch interfaces; S^0 dofs are numbered in increasing order of their
 *             lowest S^2 representative.
 *   Sound-soft problems are posed on S^2, sound-hard problems on S^0.
 */
#ifndef IGAFMM_H
#define IGAFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int igb_status;
#define IGB_OK 0
/* hip_stream value selecting the context's own stream */
#define IGB_CONTEXT_STREAM ((void*)(~(uintptr_t)0))

#define IGB_ERR_ARG (-1)       /* invalid argument                                   */
#define IGB_ERR_GEOMETRY (-2)  /* invalid knots / weights / non-conforming patches   */
#define IGB_ERR_BUDGET (-3)    /* the context's HBM budget would be exceeded          */
#define IGB_ERR_HIP (-4)       /* a HIP runtime call failed                           */
#define IGB_ERR_UNSUPPORTED (-5) /* parameters outside what the library implements    */
#define IGB_WARN_NOT_CONVERGED 1 /* iterative solve stopped at maxit                  */

typedef struct igb_ctx_s* igb_ctx;
typedef struct igb_geom_s* igb_geom;
typedef struct igb_op_s* igb_op;

/* One NURBS patch F_j: [0,1]^2 -> Gamma_j (Sec. 3.2).  Open knot vectors of
 * length ncp+deg+1 in [0,1]; cpw[ncp_v][ncp_u][4] = (x, y, z, w) with w > 0
 * (Cartesian control point and weight, not homogeneous).  Patches must be
 * oriented so that d_u F x d_v F points outward, and conform along shared edges
 * (the two patch maps agree on the interface up to a symmetry of the square). */
typedef struct {
    int deg_u, deg_v, ncp_u, ncp_v;
    const double* knots_u;
    const double* knots_v;
    const double* cpw;
} igb_patch;

typedef enum { IGB_SOFT = 0, IGB_HARD = 1 } igb_bc;
typedef enum { IGB_FP64 = 0, IGB_MIX_FP32 = 1, IGB_MIX_BF16 = 2 } igb_prec;
typedef enum {
    IGB_CFIE = 0,
    IGB_SINGLE_LAYER = 1,
    IGB_OP_V = 2,
    IGB_OP_KSTAR = 3,
    IGB_OP_K = 4,
    IGB_OP_W = 5
} igb_formulation;

/* Operator parameters.
 *   kappa      wavenumber (> 0)
 *   bc         IGB_SOFT: (1/2 M + K* - i eta V) on S^2 (Sec. 4.1, system D2N);
 *              IGB_HARD: (1/2 M - K - i eta W) on S^0 (Sec. 4.1, system N2D, W
 *              regularised as in Sec. 4.3)
 *   eta_c      CFIE coupling eta (Sec. 2, any real value != 0); 0 selects kappa (soft)
 *              and -1/kappa (hard), for which every mode of the sphere operators
 *              has a positive real part
 *   q          interpolation degree per reference direction (q+1 Chebyshev
 *              points of the first kind, Sec. 4.4), 1 <= q <= 10
 *   eta_adm    admissibility: dist(B_t,B_s) >= eta_adm * max(diam B_t, diam B_s)
 *              for the boxes of the clusters' Bezier control points (Sec. 4.4
 *              gives eta = 1.6 without the inequality; this reading), and only
 *              for clusters that each lie inside one knot span of their
 *              patch's geometry (Sec. 3.2 takes the mappings to be smooth;
 *              across a knot line the pulled-back kernel is only finitely
 *              smooth and its interpolant converges algebraically in q)
 *   kcap       if > 0, a block is admissible only if kappa*max(diam) <= kcap
 *   leaf_depth clusters stop at 4^leaf_depth elements (leaf level m - leaf_depth),
 *              0 <= leaf_depth <= 6
 *   precision  far-field coupling storage: IGB_FP64; IGB_MIX_FP32 / IGB_MIX_BF16 add
 *              couplings rounded (RNE) to fp32 / bf16 that cfie_solve uses inside
 *              iterative refinement (inner GMRES on the rounded far field with fp32
 *              accumulation on the matrix cores, outer residual in fp64) and
 *              h2_matvec uses with IGB_MV_LOWPREC; Arnoldi and residuals stay fp64,
 *              and so does the near field, except that IGB_MIX_BF16 keeps an fp32 copy
 *              that IGB_MV_LOWPREC products use (fp32 columns, products and row sums,
 *              on the matrix cores in tiles of rows over a common column list), and
 *              IGB_MIX_FP32 an fp64 copy in the same tiles that its IGB_MV_LOWPREC
 *              products use (fp64 on the matrix cores, every block size)
 *   far_on_the_fly  0: the fp64 couplings are stored ((q+1)^4 complex per far pair,
 *              two for IGB_HARD); 1: none are stored and every fp64 far-field
 *              product (fp64 matvecs, refinement residuals) evaluates the kernel at
 *              the node pairs as it goes: the same interpolated operator (to
 *              rounding), no coupling memory, bound by fp64 arithmetic
 *   quad_extra Gauss points per direction added to (negative: removed from) the
 *              default near-field rules (regular pairs: per element and direction
 *              4..12 by centre distance / extent in that direction, raised with
 *              kappa * size, at least 2 and at most 12, at most 100 points per
 *              element; touching pairs:
 *              7 / 8 / 9 for identical / edge / vertex, raised with kappa times the
 *              largest element size and with the largest element aspect ratio,
 *              at most 16); values > 0 also raise the rules of the right-hand
 *              side, far field and potential (base 6, 6 and 8, raised with
 *              kappa * element size, at most 16),
 *              -2 <= quad_extra <= 3: accuracy of the near field against assembly time
 *   formulation IGB_CFIE: the systems above (direct, Sec. 4.1); IGB_SINGLE_LAYER:
 *              the indirect single-layer ansatz u_s = -S t with t on S^2 (Sec. 5.2
 *              compares against such solutions): IGB_SOFT solves V t = <u_inc, psi>,
 *              IGB_HARD the adjoint double-layer equation (K* - 1/2 M) t =
 *              <d_n u_inc, psi>; solutions, far fields and potentials then use the
 *              sound-soft representation for both; eta_c is ignored.  Neither is
 *              uniquely solvable at the interior Dirichlet eigenvalues of kappa.
 *              IGB_OP_V / IGB_OP_KSTAR (on S^2) and IGB_OP_K / IGB_OP_W (regularised,
 *              on S^0): the single Galerkin matrix of that boundary integral operator
 *              (Sec. 4.1-4.3) as its own H^2 matrix, for h2_matvec only (cfie_rhs,
 *              cfie_solve, farfield and potential return IGB_ERR_ARG); bc is ignored
 *   separate   0: one H^2 matrix of the combined kernel (default); 1 (IGB_CFIE only):
 *              one H^2 matrix per operator as in Sec. 5.1's set-up (soft: 1/2 M + K*
 *              and V; hard: 1/2 M - K and W), each with its own near field and
 *              couplings, applied as a lazy sum; the same system up to rounding at
 *              twice the coupling memory and traffic.  igb_op_near_csr,
 *              igb_op_far_blocks, igb_op_near_pairs, igb_op_profile and
 *              igb_op_kernel_time return IGB_ERR_ARG on such an operator.
 *   far_recompress_tol  0: off.  > 0 (at most 1e-2; sound-soft family, stored fp64
 *              couplings, q <= 7): each coupling tile K is also factored by
 *              Householder QR with column pivoting, K P = Q R, truncated at the
 *              first rank k with ||R(k:, k:)||_F <= tol ||K||_F, so K ~ U W with
 *              U = Q(:, 0:k), W = R(0:k, :) P^T and ||K - U W||_F <= tol ||K||_F;
 *              the one-column fp64 products (h2_matvec with nrhs = 1,
 *              single-direction solves and residuals) then stream the factors
 *              (2 nq k complex per pair instead of nq^2).  Products of several
 *              columns keep using the tiles. */
typedef struct {
    double kappa;
    int bc;
    double eta_c;
    int q;
    double eta_adm;
    double kcap;
    int leaf_depth;
    int precision;
    int far_on_the_fly;
    int quad_extra;
    int formulation;
    int separate;
    double far_recompress_tol;
} igb_op_params;

typedef struct {
    double tol;      /* relative residual ||b - A x|| / ||b||, Euclidean on coefficients */
    int restart;     /* GMRES restart length (the paper uses 30, Sec. 5.1)              */
    int maxit;       /* maximal number of Arnoldi steps per column (over all refinements) */
    double inner_tol;/* mixed precision: lower bound of the inner relative tolerance;
                        <= 0 selects 0 (fp32) / 1e-3 (bf16)                             */
    int refine_max;  /* mixed precision: maximal refinement steps on the reduced-precision
                        operator (<= 0: 10); a column escalated to fp64 gets up to 3 more */
    int verbose;     /* 1: one line on stderr per restart cycle and refinement step
                        (Arnoldi steps, largest relative residual, elapsed seconds)   */
} igb_solve_params;

typedef struct {
    int iters;        /* Arnoldi steps (max over columns, summed over refinements)  */
    int converged;    /* number of columns that reached tol                         */
    double relres;    /* max over columns of the final recursive relative residual   */
    double relres_true; /* max over columns of ||b - A x||/||b|| recomputed at the end */
    int64_t matvecs;  /* operator applications in total (Arnoldi + residual checks) */
    int refinements;  /* mixed precision: outer refinement steps taken (all columns)  */
    int escalated;    /* mixed precision: columns that finished on the fp64 operator
                         because a refinement step reduced their fp64 residual by
                         less than a factor 10                                       */
    double seconds;   /* wall time of cfie_solve (right-hand sides, GMRES, residual
                         checks), host clock                                         */
} igb_solve_info;

typedef struct {
    int64_t n;              /* dimension of the solution space                     */
    int64_t nelem;          /* elements                                            */
    int64_t n2;             /* dim S^2                                             */
    int64_t nclusters;      /* clusters on levels 0..leaf                          */
    int leaf_level;
    int nq;                 /* (q+1)^2                                             */
    int64_t far_pairs;      /* admissible (ordered) cluster pairs, all levels       */
    int64_t far_per_level[16];
    int64_t near_elem_pairs;/* element pairs integrated by quadrature              */
    int64_t nnz;            /* nonzeros of the near-field matrix                    */
    int64_t device_bytes;   /* device memory held by the operator                   */
    int64_t estimated_bytes;/* device memory the operator holds after assembly, a
                               one-direction solve and its far field at 64 directions
                               (size model; also on host-only contexts);
                               assemble_nearfield checks the budget against this
                               plus its own transient staging buffers              */
    double assembly_near_ms, assembly_far_ms;
    int64_t far_factor_entries; /* far_recompress_tol > 0: complex entries of all tile
                                   factors (2 nq rank per far pair); else 0          */
    int64_t near_col_entries;   /* int32 column indices the one-column near product
                                   reads: one list per group of rows with the same
                                   leaves (the CSR's own indices are not read)      */
    int64_t near_tile_entries;  /* complex entries of the near field in the tile
                                   layout of the matrix-core near products (rows of a
                                   tile share one column list; missing entries are
                                   stored as zeros)                                 */
    int64_t near_group_staged;  /* 1: the one-column near product stages each row
                                   group's x entries in LDS (the longest list fits
                                   the device's LDS per workgroup); 0: it gathers x
                                   per nonzero                                      */
} igb_op_info;

/* ---------------------------------------------------------------- context */

#define IGB_HOST_ONLY (-1)
/* Creates a context on HIP device `device`, or, with device = IGB_HOST_ONLY, a
 * context without a device: geometries and operators created on it run the
 * host stages only (validation, spaces, cluster trees, block partition, near
 * pairs and sparsity pattern) and every compute entry point on them fails with
 * IGB_ERR_ARG.  hbm_budget_bytes = 0 means no
 * limit; otherwise geometry and operator creation fail with IGB_ERR_BUDGET
 * before allocating if the context would hold more.  *out receives the handle. */
igb_status igb_ctx_create(int device, size_t hbm_budget_bytes, igb_ctx* out);
void igb_ctx_destroy(igb_ctx ctx);
/* Bytes currently held by the context's geometries and operators. */
size_t igb_ctx_used_bytes(igb_ctx ctx);

/* ---------------------------------------------------------------- geometry */

/* Discretises npatch NURBS patches (host arrays, Sec. 3.2) with the spaces of
 * Sec. 3.3 at refinement level m (2^m x 2^m elements per patch) and spline
 * degree p (0 <= p <= 3; S^0 needs p >= 1).  Geometry degree per knot span must
 * be <= 3 and every geometry knot must be a mesh knot j/2^m.  Errors:
 * IGB_ERR_GEOMETRY for invalid knots, weights <= 0 or patches that do not
 * conform; IGB_ERR_ARG for bad sizes. */
igb_status build_geometry(igb_ctx ctx, const igb_patch* patches, int npatch, int level_m,
                          int degree_p, igb_geom* out);
void igb_geom_destroy(igb_geom g);
/* dims[0] = elements, dims[1] = dim S^2, dims[2] = dim S^0 (0 if p = 0). */
igb_status igb_geom_dims(igb_geom g, int64_t dims[3]);
/* The S^0 number of every S^2 dof (host array of dim S^2). */
igb_status igb_geom_s0_map(igb_geom g, int32_t* s2_to_s0);

/* ---------------------------------------------------------------- operator */

/* Assembles the CFIE operator of Sec. 4.1 with the H^2 compression of Sec. 4.4:
 * the cluster trees and block partition (host), the near-field Galerkin
 * matrix by quadrature on the device (Duffy-type singular rules on touching
 * element pairs, tensor Gauss otherwise; includes 1/2 M), and the coupling
 * matrices of every admissible block on the device.  Synchronous. */
igb_status assemble_nearfield(igb_ctx ctx, igb_geom g, const igb_op_params* prm, igb_op* out);
void igb_op_destroy(igb_op op);
igb_status igb_op_get_info(igb_op op, igb_op_info* info);
/* Dimension N of the solution space (dim S^2 soft, dim S^0 hard); -1 for NULL. */
int64_t igb_op_ndof(igb_op op);
/* Device bytes the operator holds now (data and grown work buffers); -1 for NULL. */
int64_t igb_op_bytes(igb_op op);

/* Size model of a solve: *bytes = device memory the operator holds after
 * cfie_solve with ndir directions and GMRES restart `restart` (0 = 30) and the
 * far field of those ndir columns at up to 64 directions: its data
 * (estimated_bytes of igb_op_info without the one-column work), the matvec work
 * vectors of ndir columns, the solver's buffers (Krylov bases, right-hand
 * sides, refinement residual and corrections) and the right-hand-side and
 * far-field quadrature buffers.  cfie_solve checks the budget
 * against this model before any work and returns IGB_ERR_BUDGET if the growth
 * would not fit.  Works on host-only contexts (admission planning). */
igb_status igb_op_solve_bytes(igb_op op, int ndir, int restart, int64_t* bytes);

/* Near-field matrix in CSR (solution space) copied to host arrays of sizes
 * n+1, nnz, 2*nnz (sizes from igb_op_get_info). */
igb_status igb_op_near_csr(igb_op op, int64_t* row_ptr, int32_t* col, double* val);
/* Admissible blocks: out[4*i..] = (level, target, source, 0) with cluster
 * indices local to the level: patch*4^l + cy*2^l + cx. */
igb_status igb_op_far_blocks(igb_op op, int32_t* out);

/* Near element pairs (host arrays): ptr[nelem+1], src[near_elem_pairs] sorted per
 * target element, kind[near_elem_pairs] = quadrature class (bits 0-3: 0 regular,
 * 1 common vertex, 2 common edge, 4 identical; regular pairs: bits 8-11 /
 * 12-15 Gauss orders along u / v on the test element, bits 16-19 / 20-23 on
 * the trial element; touching pairs: bits 16-18 / 20-22 square symmetries
 * bringing the pair into the canonical configuration).  Works on host-only
 * contexts. */
igb_status igb_op_near_pairs(igb_op op, int64_t* ptr, int32_t* src, int32_t* kind);

/* Per-kernel timing with HIP events recorded on the launch stream around the
 * operator's matvec stages: "m2l" (coupling), "spmv" (near field + combine),
 * "upward" (leaf moments + transfers up), "downward" (reduce, transfers down,
 * back projection).  igb_op_profile(op, 1) starts recording (and clears);
 * igb_op_kernel_time waits for the recorded launches and returns their count
 * and total milliseconds, then clears that kernel's record. */
igb_status igb_op_profile(igb_op op, int enable);
igb_status igb_op_kernel_time(igb_op op, const char* name, int64_t* launches, double* total_ms);

/* HIP graphs for the matvec (off by default): with enable = 1, each distinct
 * (x, y, nrhs, parts, stream) of h2_matvec and of the matvecs inside
 * cfie_solve is captured once from a non-null stream into a HIP graph of
 * kernel launches and replayed afterwards, which removes the host launch cost
 * of the ~20 kernels per application.  Capture puts the stream in capture
 * mode for the length of one launch sequence: enable it only while no other
 * host thread of the process issues work to the null stream or synchronous
 * copies (HIP refuses those during a capture).  Captures are dropped when the
 * operator's work buffers grow and when graphs are disabled. */
igb_status igb_op_use_graphs(igb_op op, int enable);

/* Tile shapes of the block kernels (a tuning knob; results do not change):
 * coupling_col_tiles = 16-column tiles each workgroup of the fp64 matrix-core
 * coupling carries (every tile value read serves that many column tiles),
 * near_col_tiles = the same for the fp64 matrix-core near product; 1, 2 or 4,
 * or 0 for the automatic choice (coupling: the widest that keeps at least 512
 * workgroups; near product: 2 where that keeps 512 workgroups, else 1).  A value that does not divide a block's column tile count
 * falls back to the automatic choice for that block.  Every column's result
 * is bitwise the same for every shape.  Drops the operator's captured graphs.
 * IGB_ERR_ARG for other values. */
igb_status igb_op_set_tile_shape(igb_op op, int coupling_col_tiles, int near_col_tiles);

#define IGB_PART_NEAR 1
#define IGB_PART_FAR 2
#define IGB_PART_ALL 3
#define IGB_MV_LOWPREC 4   /* with IGB_MIX_* operators: far field from the rounded copy */
#define IGB_MV_HOST 8      /* x and y are host arrays; the call is synchronous          */
/* y = A x for nrhs columns (device arrays [nrhs][n] complex; with IGB_MV_HOST in
 * parts, host arrays: x is copied to operator-owned device buffers, the product
 * runs on hip_stream, y is copied back and the call returns when y is written --
 * the timing then includes the PCIe copies).  parts selects the
 * near-field (incl. 1/2 M) and/or far-field (H^2) contributions.  The columns
 * share every pass over the couplings and the near-field matrix.  Batch
 * invariance: a column's result does not depend on the other columns, with one
 * exception -- IGB_FP64 operators with stored couplings, and the fp64 far field
 * of sound-hard operators evaluated on the fly (far_on_the_fly, any precision),
 * run the coupling of blocks of 16 or more columns on the fp64 matrix cores,
 * which sum the same products in another order than the single-column vector
 * kernels.  Results of
 * blocks of 1..15 columns are bitwise equal to single-column results, results of
 * blocks of >= 16 columns bitwise equal to those of any other block of >= 16,
 * and the two differ by rounding (<= 1e-12 relative to max|y| of the column;
 * ~1e-15 measured).  Operators with far_recompress_tol > 0 apply the tile
 * factors to single columns and the tiles to blocks of 2 or more: a column
 * alone and the same column in a block differ by the truncation, at most
 * far_recompress_tol ||K||_F per tile (2e-10 relative to max|y| measured at
 * 1e-8 on the level-5 sphere); blocks of 2..15 columns agree bitwise with each
 * other.  Reduced-precision products (IGB_MV_LOWPREC) use the matrix cores for
 * every block size and are batch invariant bitwise.  x and y must not overlap.
 * Stream-ordered. */
igb_status h2_matvec(igb_op op, const double* x, double* y, int nrhs, int parts, void* hip_stream);

/* Allocation-free variant of h2_matvec, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, layout and results as h2_matvec (device arrays
 * only: IGB_MV_HOST is rejected), computed by the same kernels, but the matvec
 * work buffers (cluster moments, coupling partials, rounded source vectors,
 * far-field result) are carved out of one static device array of
 * IGB_NOALLOC_SCRATCH_BYTES per GPU, which every context creation on that GPU
 * locates once and which the process holds until it ends.  The call allocates
 * nothing (no hipMalloc, no library routine that allocates) and uses no HIP
 * graph.  Limits and errors: IGB_ERR_ARG if the work buffers of nrhs columns
 * exceed the scratch (e.g. the level-5 sphere at q = 6 fits 16 fp64 columns),
 * if per-kernel profiling is enabled on the operator, or for invalid
 * arguments; IGB_ERR_UNSUPPORTED for operators stored as separate H^2
 * matrices.  Every call on one GPU shares that GPU's scratch (it keeps the last
 * call's contents; nothing in it needs to start at zero): calls that overlap on
 * one GPU -- on different streams, or from different host threads without
 * ordering -- race and give wrong results.  Stream-ordered like h2_matvec. */
#define IGB_NOALLOC_SCRATCH_BYTES (256u << 20)
igb_status h2_matvec_noalloc(igb_op op, const double* x, double* y, int nrhs, int parts, void* hip_stream);

/* Right-hand sides (Sec. 4.1 load vectors of the D2N / N2D systems) for ndir
 * incident plane waves e^{i kappa <d,x>} (host dirs [ndir][3], normalised here;
 * error if |d| < 1e-12) into the device array b [ndir][n].  Stream-ordered. */
igb_status cfie_rhs(igb_op op, const double* dirs, int ndir, double* b, void* hip_stream);

/* Solves the CFIE for ndir incident directions (host dirs [ndir][3]) with
 * restarted GMRES (Sec. 5.1), x0 = 0, writing the coefficients into the device
 * array coeffs [ndir][n].  The directions run in lockstep: one block matvec per
 * Arnoldi step, each column with its own Krylov basis, rotations and stopping
 * test, so a column's solution does not depend on the other columns (with the
 * exceptions stated at h2_matvec: IGB_FP64 operators with stored couplings solve
 * ndir >= 16 with matrix-core couplings, whose iterates differ from those of
 * smaller batches by rounding, as do the fp64 residuals of sound-hard
 * operators with the far field on the fly, and recompressed operators solve one direction
 * with the tile factors and several with the tiles; within each range the
 * iterates agree bitwise).
 * Operators with IGB_MIX_* precision solve by iterative refinement:
 * x += GMRES(A_rounded, b - A_fp64 x) until the fp64 residual reaches tol; a
 * column whose step reduces that residual by less than a factor 10 continues
 * with GMRES(A_fp64, .) (a step that does not reduce it is taken back first).
 * Synchronous.  IGB_WARN_NOT_CONVERGED if a column stops at maxit. */
igb_status cfie_solve(igb_op op, const double* dirs, int ndir, const igb_solve_params* sp,
                      double* coeffs, igb_solve_info* info);

/* Far-field pattern u_inf (Sec. 1) of the scattered wave for ndir coefficient
 * columns (device coeffs [ndir][n]) at nobs unit directions (host obs
 * [nobs][3]) into the device array uinf [ndir][nobs].  Sound-soft:
 * u_inf(x) = -(1/4pi) int e^{-i kappa x.y} t(y); sound-hard:
 * u_inf(x) = -(i kappa/4pi) int (x.n_y) e^{-i kappa x.y} g(y).  Stream-ordered. */
igb_status farfield(igb_op op, const double* coeffs, int ndir, const double* obs, int nobs,
                    double* uinf, void* hip_stream);

/* Scattered field at points off the boundary (the representation formulas of
 * Sec. 2 with the potentials' signs read as u = u_inc + u_s, u_s = -V t for
 * IGB_SOFT and u_s = D g for IGB_HARD):
 *   soft  u_s(x) = -int G(x,y) t(y) dsigma_y,
 *   hard  u_s(x) =  int dG(x,y)/dn_y g(y) dsigma_y,   G = e^{i kappa r}/(4 pi r),
 * for ndir coefficient vectors (device coeffs [ndir][n]) at npts points (host
 * points [npts][3]) into device u [ndir][npts], by tensor Gauss quadrature
 * on every element (8 x 8 points, more for elements large against the
 * wavelength or quad_extra > 0).  Accurate for points at least about one
 * element diameter from the surface (no near-singular correction is applied
 * closer in).  IGB_ERR_ARG for non-finite points.  Synchronous. */
igb_status potential(igb_op op, const double* coeffs, int ndir, const double* points, int npts, double* u,
                     void* hip_stream);

/* The same scattered field evaluated with an H^2 structure on the operator's
 * geometry, with its q, eta_adm and kcap (Sec. 4.4's interpolation applied to
 * the representation formula, Sec. 2):
 * the points are sorted into the boxes of an octree (at most 128 points each);
 * the sources are the patch quadtrees down to clusters of 4 elements (level
 * max(m - 1, 0), whatever the operator's leaf depth), with the moments of the
 * density on the (q+1)^2 tensor Chebyshev nodes of each cluster's parameter
 * square.  A source cluster acts through its moments at its interpolation
 * nodes when it is admissible for a box: distance at least the operator's
 * eta_adm times the cluster's diameter (boxes of the points and of the
 * cluster's control points) and kappa * diam at most the operator's kcap, or
 * q/2 if kcap is 0.  Where the box holds more points than the (q+1)^3 tensor
 * Chebyshev nodes of its own box, and the pair is admissible with the box's
 * diameter too, the nodes' kernel values are summed on the box's nodes and
 * interpolated to the points; otherwise they are summed at the points
 * directly.  The elements of the box's inadmissible 4-element clusters are summed
 * directly as in potential().  Error against potential(): the interpolation
 * error of q on the cluster side (and the box side where its nodes are
 * used).  Arguments, layout, ownership and errors
 * as for potential(), and IGB_ERR_ARG if a box list outgrows 2^31 entries
 * (hundreds of millions of points: pass them in parts); its buffers are its
 * own, allocated and freed by the call.  Synchronous. */
igb_status potential_h2(igb_op op, const double* coeffs, int ndir, const double* points, int npts, double* u,
                        void* hip_stream);

/* The plan potential_h2 builds for these points (Sec. 4.4's block partition
 * between the points' octree boxes and the source clusters), made on the host
 * alone; works on host-only contexts.  counts (4 entries, required): boxes,
 * (box, cluster) pairs summed on the box's nodes, (box, cluster) pairs summed
 * at the points through the cluster's nodes, and (box, 4-element cluster)
 * pairs summed directly.  perm (npts entries) and box_ptr (counts[0] + 1
 * entries), each optional (NULL): the points in box order (box b holds the
 * points perm[box_ptr[b]] .. perm[box_ptr[b+1] - 1], boxes in depth-first
 * octant order), so a caller sizing box_ptr calls once with it NULL.  Host
 * arrays owned by the caller.  IGB_ERR_ARG for NULL op, points or counts,
 * npts < 1, a non-finite point or lists beyond 2^31 entries, as for
 * potential_h2. */
igb_status igb_op_potential_plan(igb_op op, const double* points, int npts, int64_t* counts, int32_t* perm,
                                 int32_t* box_ptr);

const char* igb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IGAFMM_H */

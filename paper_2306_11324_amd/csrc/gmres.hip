// Restarted GMRES (Sec. 5.1: GMRES with restart 30 on the CFIE systems) on the
// device, for one or many right-hand sides in lockstep.  Arnoldi with classical
// Gram-Schmidt applied twice (CGS2); all vectors stay on the device, only the
// new Hessenberg columns (<= restart+1 complex numbers per right-hand side) go
// to pinned host memory per iteration for the Givens rotations.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <vector>

#include "common.h"

namespace igb {

namespace {

constexpr int RT = 256;

using cplx = std::complex<double>;

// progress lines of a verbose solve (stderr)
struct SolveLog {
    bool on = false;
    const char* phase = "";
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double elapsed() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

}  // namespace

namespace {

// ---- multi-column Arnoldi kernels: vectors [C][n], basis [j][C][n] ----
// Inner products in two passes: partial sums over segments of DOT_SEG entries,
// one workgroup per (jj, segment, r), then the segments summed in order
// (by cmaxpy_fin, which uses them).
constexpr int DOT_SEG = 1024;
__global__ __launch_bounds__(RT) void cdots_seg(const double2* V, int64_t n, int C, int nseg, const double2* w,
                                                double2* part) {
    __shared__ double2 red[RT];
    const int jj = blockIdx.x, sg = blockIdx.y, r = blockIdx.z;
    const double2* v = V + (int64_t(jj) * C + r) * n;
    const double2* x = w + int64_t(r) * n;
    double2 acc = make_double2(0, 0);
    const int64_t i1 = min(n, int64_t(sg + 1) * DOT_SEG);
    for (int64_t i = int64_t(sg) * DOT_SEG + threadIdx.x; i < i1; i += RT) {
        const double2 a = v[i], b = x[i];
        acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
        acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = RT / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            red[threadIdx.x].x += red[threadIdx.x + st].x;
            red[threadIdx.x].y += red[threadIdx.x + st].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t(jj) * C + r) * nseg + sg] = red[0];
}

// w[r][i] -= sum_jj h[jj*C + r] V[jj][r][i], with h the dot products summed from
// their segment partials (in segment order) by each workgroup for the columns
// its 64 entries touch (64 / n + 2 at most); the workgroup holding a column's
// first entry also stores that column's h for the host.
__global__ __launch_bounds__(64) void cmaxpy_fin(const double2* V, int nvec, int64_t n, int C, const double2* part,
                                                 int nseg, double2* h, double2* w) {
    extern __shared__ double2 hs[];   // [columns touched][nvec]
    const int64_t g0 = int64_t(blockIdx.x) * 64;
    const int rlo = int(g0 / n);
    const int rhi = int(min(g0 + 63, n * C - 1) / n);
    for (int t = threadIdx.x; t < (rhi - rlo + 1) * nvec; t += 64) {
        const int r = rlo + t / nvec, jj = t % nvec;
        double2 acc = make_double2(0, 0);
        for (int sg = 0; sg < nseg; ++sg) {
            const double2 v = part[(int64_t(jj) * C + r) * nseg + sg];
            acc.x += v.x;
            acc.y += v.y;
        }
        hs[t] = acc;
        if (int64_t(r) * n >= g0 && int64_t(r) * n < g0 + 64) h[int64_t(jj) * C + r] = acc;
    }
    __syncthreads();
    const int64_t gid = g0 + threadIdx.x;
    if (gid >= n * C) return;
    const int r = int(gid / n);
    const int64_t i = gid % n;
    const double2* hc = hs + (r - rlo) * nvec;
    double2 acc = w[gid];
    for (int j = 0; j < nvec; ++j) {
        const double2 a = hc[j], v = V[(int64_t(j) * C + r) * n + i];
        acc.x -= a.x * v.x - a.y * v.y;
        acc.y -= a.x * v.y + a.y * v.x;
    }
    w[gid] = acc;
}

// x[r][i] += sum_jj y[jj*C + r] V[jj][r][i]
__global__ void cupdate_multi(const double2* V, int nvec, int64_t n, int C, const double2* y, double2* x) {
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= n * C) return;
    const int r = int(gid / n);
    const int64_t i = gid % n;
    double2 acc = x[gid];
    for (int j = 0; j < nvec; ++j) {
        const double2 a = y[int64_t(j) * C + r], v = V[(int64_t(j) * C + r) * n + i];
        acc.x += a.x * v.x - a.y * v.y;
        acc.y += a.x * v.y + a.y * v.x;
    }
    x[gid] = acc;
}

// out[r] = ||w[r]||^2, one workgroup per column
__global__ __launch_bounds__(1024) void cnorm2_multi(const double2* w, int64_t n, double* out) {
    __shared__ double red[1024];
    const double2* x = w + int64_t(blockIdx.x) * n;
    double acc = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) acc = fma(x[i].x, x[i].x, fma(x[i].y, x[i].y, acc));
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// out[r] = ||w[r]||^2 and v[r][i] = w[r][i] / sqrt(out[r]) (0 for a zero
// column), one workgroup per column: the next Arnoldi vector, normalised on the
// device so that no scale factors travel per step (the norm's sums are those of
// cnorm2_multi)
__global__ __launch_bounds__(1024) void cnorm_scale(const double2* w, int64_t n, double* out, double2* v) {
    __shared__ double red[1024];
    const double2* x = w + int64_t(blockIdx.x) * n;
    double acc = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) acc = fma(x[i].x, x[i].x, fma(x[i].y, x[i].y, acc));
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double q = red[0];
    if (threadIdx.x == 0) out[blockIdx.x] = q;
    const double f = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    double2* y = v + int64_t(blockIdx.x) * n;
    for (int64_t i = threadIdx.x; i < n; i += 1024) y[i] = make_double2(x[i].x * f, x[i].y * f);
}

// v[r][i] = w[r][i] * sc[r]
__global__ void cscale_multi(const double2* w, int64_t n, int C, const double* sc, double2* v) {
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= n * C) return;
    const double f = sc[gid / n];
    v[gid] = make_double2(w[gid].x * f, w[gid].y * f);
}

// r = b - r ; x += d ; zero columns
__global__ void csub_from_multi(const double2* b, int64_t nc, double2* r) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nc) r[i] = make_double2(b[i].x - r[i].x, b[i].y - r[i].y);
}
__global__ void cadd_to(const double2* d, int64_t nc, double2* x) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nc) x[i] = make_double2(x[i].x + d[i].x, x[i].y + d[i].y);
}

struct ColumnResult {
    int iters = 0;
    int64_t applications = 0;
    bool converged = false;
    double relres = 1.0;      // recursive estimate at exit
    double true_rel = 1.0;    // ||B - A X|| / ||B|| recomputed with the same operator
};

struct Work {
    int64_t n;
    int m, C, nseg;
    double2 *V, *w, *r, *R, *D, *h, *h2, *y, *part;
    double *nrm, *sc;
    double2* hp[2];      // pinned coherent host buffers that the kernels of alternate steps write
                         // h, h2 and the squared norms into
    hipEvent_t ev[2];    // the step writing hp[k] has finished
};

struct SolveSizes {
    size_t krylov, w, h, dotpart, rhs, ref;   // ref: each of the three refinement buffers
};
SolveSizes solve_sizes(const igb_op_s* op, int m, int C) {
    const size_t n = size_t(op->N);
    const size_t nseg = (n + DOT_SEG - 1) / DOT_SEG;
    SolveSizes z;
    z.krylov = size_t(m + 1) * C * n * sizeof(double2);
    z.w = size_t(4) * C * n * sizeof(double2);
    z.h = size_t(3) * (m + 2) * C * sizeof(double2) + size_t(2) * C * sizeof(double) + 64;
    z.dotpart = size_t(m + 1) * C * nseg * sizeof(double2);
    z.rhs = size_t(C) * n * sizeof(double2);
    z.ref = op->prm.precision != IGB_FP64 ? size_t(C) * n * sizeof(double2) : 0;
    return z;
}

igb_status ensure_work(igb_op op, int m, int C, Work& W) {
    const int64_t n = op->N;
    const SolveSizes z = solve_sizes(op, m, C);
    const size_t need_h = z.h;
    // the budget check covers the whole growth before anything is released
    igb_ctx ctx = op->geom->ctx;
    size_t grow_by = 0;
    for (auto bs : {std::make_pair(&op->d_krylov, z.krylov), std::make_pair(&op->d_w, z.w),
                    std::make_pair(&op->d_h, z.h), std::make_pair(&op->d_dotpart, z.dotpart)})
        grow_by += bs.first->bytes >= bs.second ? 0 : bs.second - bs.first->bytes;
    if (ctx->budget != 0 && ctx->used.load() + grow_by > ctx->budget) {
        set_error("cfie_solve: HBM budget exceeded by the Krylov bases of %d columns (%zu held + %zu > %zu bytes)", C,
                  ctx->used.load(), grow_by, ctx->budget);
        return IGB_ERR_BUDGET;
    }
    igb_status st;
    const int nseg = int((n + DOT_SEG - 1) / DOT_SEG);
    if ((st = op_reserve(op, op->d_krylov, z.krylov, "cfie_solve")) || (st = op_reserve(op, op->d_w, z.w, "cfie_solve")) ||
        (st = op_reserve(op, op->d_h, z.h, "cfie_solve")) ||
        (st = op_reserve(op, op->d_dotpart, z.dotpart, "cfie_solve")))
        return st;
    W.nseg = nseg;
    W.part = op->d_dotpart.as<double2>();
    W.n = n;
    W.m = m;
    W.C = C;
    W.V = op->d_krylov.as<double2>();
    W.w = op->d_w.as<double2>();
    W.r = W.w + int64_t(C) * n;
    W.R = W.r + int64_t(C) * n;
    W.D = W.R + int64_t(C) * n;
    // h, h2 and the squared norms are contiguous: one copy to the host per Arnoldi step
    W.h = op->d_h.as<double2>();
    W.h2 = W.h + int64_t(m + 2) * C;
    W.nrm = reinterpret_cast<double*>(W.h2 + int64_t(m + 2) * C);
    W.sc = W.nrm + C;
    W.y = reinterpret_cast<double2*>(W.sc + C);
    if (op->h_pin_bytes < 2 * need_h) {
        if (op->h_pin) (void)hipHostFree(op->h_pin);
        op->h_pin = nullptr;
        op->h_pin_bytes = 0;
        IGB_HIP(hipHostMalloc(&op->h_pin, 2 * need_h, hipHostMallocCoherent));
        op->h_pin_bytes = 2 * need_h;
    }
    W.hp[0] = static_cast<double2*>(op->h_pin);
    W.hp[1] = reinterpret_cast<double2*>(static_cast<char*>(op->h_pin) + need_h);   // need_h is a multiple of 16
    for (int k = 0; k < 2; ++k) {
        if (!op->ev_h[k]) IGB_HIP(hipEventCreateWithFlags(&op->ev_h[k], hipEventDisableTiming));
        W.ev[k] = op->ev_h[k];
    }
    return IGB_OK;
}

igb_status norms(const double2* v, int64_t n, int C, double* dev_tmp, std::vector<double>& out, hipStream_t s) {
    hipLaunchKernelGGL(cnorm2_multi, dim3(C), dim3(1024), 0, s, v, n, dev_tmp);
    out.resize(C);
    IGB_HIP(hipMemcpyAsync(out.data(), dev_tmp, C * sizeof(double), hipMemcpyDeviceToHost, s));
    IGB_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < C; ++r) out[r] = std::sqrt(out[r]);
    return IGB_OK;
}

// Lockstep restarted GMRES for C columns: every column runs its own Arnoldi
// process and Givens rotations; the operator is applied to all columns at once.
// X = 0 initially; column c stops when its recursive relative residual reaches
// tol[c] (or after maxit[c] Arnoldi steps).  Columns never interact; the block
// matvec always covers all C columns, so a column's iterates depend on the batch
// only through the matvec's code path: fp64 operators with stored couplings
// take the matrix-core coupling for C >= 16 (another summation order, equal to
// the vector path up to rounding), recompressed operators the tile factors for
// C = 1 and the tiles for C >= 2 (equal up to the truncation); every other
// case is bitwise batch invariant.
igb_status gmres_block(igb_op op, const Work& Wk, const double2* B, double2* X, const std::vector<int>& maxit,
                       const std::vector<double>& tol, int mvflags, hipStream_t s, std::vector<ColumnResult>& res,
                       const SolveLog& log) {
    const int64_t n = Wk.n;
    const int m = Wk.m, C = Wk.C;
    const unsigned gb = unsigned((n * C + 255) / 256);
    const unsigned gb64 = unsigned((n * C + 63) / 64);
    double2 *V = Wk.V, *w = Wk.w, *r = Wk.r;
    igb_status st;
    IGB_HIP(hipMemsetAsync(X, 0, n * C * sizeof(double2), s));
    std::vector<double> bnorm, rnorm, hn;
    if ((st = norms(B, n, C, Wk.nrm, bnorm, s))) return st;
    res.assign(C, ColumnResult());
    for (int c = 0; c < C; ++c) {
        res[c].converged = bnorm[c] == 0.0;
        res[c].relres = res[c].true_rel = res[c].converged ? 0.0 : 1.0;
    }
    IGB_HIP(hipMemcpyAsync(r, B, n * C * sizeof(double2), hipMemcpyDeviceToDevice, s));
    rnorm = bnorm;
    std::vector<std::vector<cplx>> H(C, std::vector<cplx>(size_t(m + 1) * m)), cs(C, std::vector<cplx>(m)),
        sn(C, std::vector<cplx>(m)), g(C, std::vector<cplx>(m + 1));
    std::vector<double2> yd;
    std::vector<double> sc(C);
    std::vector<int> jc(C);
    auto active = [&](int c) { return !res[c].converged && res[c].iters < maxit[c]; };
    for (;;) {
        bool any = false;
        for (int c = 0; c < C; ++c) any = any || active(c);
        if (!any) break;
        // start a cycle: V_0 = r / ||r|| for the active columns
        std::vector<bool> in_cycle(C);
        for (int c = 0; c < C; ++c) {
            in_cycle[c] = active(c);
            sc[c] = in_cycle[c] ? 1.0 / rnorm[c] : 0.0;
            std::fill(g[c].begin(), g[c].end(), cplx(0));
            g[c][0] = rnorm[c];
            jc[c] = 0;
        }
        IGB_HIP(hipMemcpyAsync(Wk.sc, sc.data(), C * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(cscale_multi, dim3(gb), dim3(256), 0, s, r, n, C, Wk.sc, V);
        // A column takes part in step jj if, after step jj - 1, it is in the cycle,
        // has taken jj steps and is still active.  Step j is enqueued before the
        // host processes step j - 1 (the device runs step j meanwhile, its
        // Hessenberg entries go to the other pinned buffer); if step j - 1 ends
        // every column, step j is dropped unprocessed (and not counted).
        auto going = [&](int jj) {
            for (int c = 0; c < C; ++c)
                if (in_cycle[c] && jc[c] == jj && active(c)) return true;
            return false;
        };
        auto enqueue = [&](int jj) -> igb_status {
            igb_status st2;
            if ((st2 = matvec_device(op, reinterpret_cast<const double*>(V + int64_t(jj) * C * n),
                                     reinterpret_cast<double*>(w), C, mvflags, s)))
                return st2;
            // classical Gram-Schmidt, twice
            const size_t hlds = size_t(std::min<int64_t>(C, 63 / n + 2)) * (jj + 1) * sizeof(double2);
            hipLaunchKernelGGL(cdots_seg, dim3(jj + 1, Wk.nseg, C), dim3(RT), 0, s, V, n, C, Wk.nseg, w, Wk.part);
            // the Hessenberg entries and the norm go straight into the step's pinned
            // host buffer (device-visible, coherent): no copy per step
            double2* hh = Wk.hp[jj & 1];
            hipLaunchKernelGGL(cmaxpy_fin, dim3(gb64), dim3(64), hlds, s, V, jj + 1, n, C, Wk.part, Wk.nseg, hh, w);
            hipLaunchKernelGGL(cdots_seg, dim3(jj + 1, Wk.nseg, C), dim3(RT), 0, s, V, n, C, Wk.nseg, w, Wk.part);
            hipLaunchKernelGGL(cmaxpy_fin, dim3(gb64), dim3(64), hlds, s, V, jj + 1, n, C, Wk.part, Wk.nseg,
                               hh + int64_t(m + 2) * C, w);
            // ||w||^2 (to the host buffer) and the next basis vector on the device
            hipLaunchKernelGGL(cnorm_scale, dim3(C), dim3(1024), 0, s, w, n,
                               reinterpret_cast<double*>(hh + int64_t(2) * (m + 2) * C), V + int64_t(jj + 1) * C * n);
            IGB_HIP(hipGetLastError());
            IGB_HIP(hipEventRecord(Wk.ev[jj & 1], s));
            return IGB_OK;
        };
        auto process = [&](int jj) -> igb_status {
            IGB_HIP(hipEventSynchronize(Wk.ev[jj & 1]));
            const double2* hp1 = Wk.hp[jj & 1];
            const double2* hp2 = hp1 + int64_t(m + 2) * C;
            const double* hpn = reinterpret_cast<const double*>(hp1 + int64_t(2) * (m + 2) * C);
            hn.resize(C);
            for (int c = 0; c < C; ++c) hn[c] = std::sqrt(hpn[c]);
            for (int c = 0; c < C; ++c) {
                if (!(in_cycle[c] && jc[c] == jj && active(c))) continue;
                ++res[c].iters;
                ++res[c].applications;
                std::vector<cplx>& Hc = H[c];
                for (int i = 0; i <= jj; ++i) {
                    const double2 a1 = hp1[size_t(i) * C + c], a2 = hp2[size_t(i) * C + c];
                    Hc[size_t(i) * m + jj] = cplx(a1.x + a2.x, a1.y + a2.y);
                }
                Hc[size_t(jj + 1) * m + jj] = hn[c];
                for (int i = 0; i < jj; ++i) {
                    cplx a = Hc[size_t(i) * m + jj], bb = Hc[size_t(i + 1) * m + jj];
                    Hc[size_t(i) * m + jj] = cs[c][i] * a + sn[c][i] * bb;
                    Hc[size_t(i + 1) * m + jj] = -std::conj(sn[c][i]) * a + cs[c][i] * bb;
                }
                cplx a = Hc[size_t(jj) * m + jj], bb = Hc[size_t(jj + 1) * m + jj];
                const double rr = std::sqrt(std::norm(a) + std::norm(bb));
                if (rr == 0) {
                    cs[c][jj] = 1;
                    sn[c][jj] = 0;
                } else if (std::abs(a) == 0) {
                    cs[c][jj] = 0;
                    sn[c][jj] = std::conj(bb) / rr;
                } else {
                    cs[c][jj] = std::abs(a) / rr;
                    sn[c][jj] = (a / std::abs(a)) * std::conj(bb) / rr;
                }
                Hc[size_t(jj) * m + jj] = cs[c][jj] * a + sn[c][jj] * bb;
                Hc[size_t(jj + 1) * m + jj] = 0;
                g[c][jj + 1] = -std::conj(sn[c][jj]) * g[c][jj];
                g[c][jj] = cs[c][jj] * g[c][jj];
                res[c].relres = std::abs(g[c][jj + 1]) / bnorm[c];
                jc[c] = jj + 1;
                if (res[c].relres <= tol[c] || hn[c] == 0) res[c].converged = true;
            }
            return IGB_OK;
        };
        int pend = -1;   // step enqueued, not yet processed
        for (int j = 0;; ++j) {
            // exact when nothing is pending; otherwise step j may run if some
            // column takes part in the pending step
            const bool enq = j < m && going(pend < 0 ? j : pend);
            if (enq && (st = enqueue(j))) return st;
            if (pend >= 0 && (st = process(pend))) return st;
            if (!enq) break;
            pend = j;
        }
        // X += V y per column (zeros beyond a column's own step count)
        int jmax = 0;
        for (int c = 0; c < C; ++c) jmax = std::max(jmax, in_cycle[c] ? jc[c] : 0);
        yd.assign(size_t(std::max(jmax, 1)) * C, make_double2(0, 0));
        for (int c = 0; c < C; ++c) {
            if (!in_cycle[c]) continue;
            const int jj = jc[c];
            std::vector<cplx> y(jj);
            for (int i = jj - 1; i >= 0; --i) {
                cplx acc = g[c][i];
                for (int kk = i + 1; kk < jj; ++kk) acc -= H[c][size_t(i) * m + kk] * y[kk];
                y[i] = acc / H[c][size_t(i) * m + i];
            }
            for (int i = 0; i < jj; ++i) yd[size_t(i) * C + c] = make_double2(y[i].real(), y[i].imag());
        }
        if (jmax > 0) {
            IGB_HIP(hipMemcpyAsync(Wk.y, yd.data(), size_t(jmax) * C * sizeof(double2), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(cupdate_multi, dim3(gb), dim3(256), 0, s, V, jmax, n, C, Wk.y, X);
        }
        // residual of the same operator: r = B - A X
        if ((st = matvec_device(op, reinterpret_cast<const double*>(X), reinterpret_cast<double*>(r), C, mvflags, s)))
            return st;
        hipLaunchKernelGGL(csub_from_multi, dim3(gb), dim3(256), 0, s, B, n * C, r);
        IGB_HIP(hipGetLastError());
        if ((st = norms(r, n, C, Wk.nrm, rnorm, s))) return st;
        int nact = 0, steps = 0;
        double worst = 0;
        for (int c = 0; c < C; ++c) {
            if (!in_cycle[c]) continue;
            ++res[c].applications;
            res[c].true_rel = bnorm[c] > 0 ? rnorm[c] / bnorm[c] : 0.0;
            ++nact;
            steps = std::max(steps, res[c].iters);
            worst = std::max(worst, res[c].true_rel);
        }
        if (log.on)
            fprintf(stderr, "[igafmm] %s cycle: %d columns, %d Arnoldi steps, largest relative residual %.2e, %.1f s\n",
                    log.phase, nact, steps, worst, log.elapsed());
    }
    return IGB_OK;
}

}  // namespace

size_t solve_buffer_bytes(const igb_op_s* op, int m, int ndir) {
    const SolveSizes z = solve_sizes(op, m, ndir);
    return z.krylov + z.w + z.h + z.dotpart + z.rhs + 3 * z.ref;
}

size_t solve_model_bytes(const igb_op_s* op, int m, int ndir, int nobs) {
    size_t b = solve_buffer_bytes(op, m, ndir) + quad_buffer_bytes(op, ndir, nobs);
    if (op->sum_parts.empty()) return b + op->estimated_data + work_sizes(op, ndir).total();
    for (const igb_op_s* p : op->sum_parts) b += p->estimated_data + work_sizes(p, ndir).total();
    return b + size_t(ndir) * op->N * sizeof(double2);   // the lazy sum's column buffer
}

igb_status gmres_device(igb_op op, const double* b_in, double* x_out, int ndir, const igb_solve_params* sp,
                        igb_solve_info* info, hipStream_t s) {
    const int64_t n = op->N;
    const int m = sp->restart > 0 ? sp->restart : 30;
    const int maxit = sp->maxit > 0 ? sp->maxit : 1000;
    const double tol = sp->tol > 0 ? sp->tol : 1e-8;
    const bool mixed = op->prm.precision != IGB_FP64;
    const int C = ndir;
    SolveLog log;
    log.on = sp->verbose != 0;
    Work W;
    igb_status st;
    if ((st = ensure_work(op, m, C, W))) return st;
    const unsigned gb = unsigned((n * C + 255) / 256);
    const double2* B = reinterpret_cast<const double2*>(b_in);
    double2* X = reinterpret_cast<double2*>(x_out);
    std::vector<ColumnResult> res;
    igb_solve_info out{};
    if (!mixed) {
        log.phase = "fp64";
        if ((st = gmres_block(op, W, B, X, std::vector<int>(C, maxit), std::vector<double>(C, tol), IGB_PART_ALL, s,
                              res, log)))
            return st;
    } else {
        // iterative refinement: inner GMRES on the reduced-precision far field,
        // outer residual with the fp64 operator; columns refine independently.
        // A column whose fp64 residual falls by less than ESCALATE per step (or
        // rises: that correction is taken back) refines from then on with the
        // fp64 operator, solving straight to the tolerance.
        const double ESCALATE = 0.1;
        const double inner_min = sp->inner_tol > 0 ? sp->inner_tol : (op->prm.precision == IGB_MIX_FP32 ? 0.0 : 1e-3);
        const int refine_max = sp->refine_max > 0 ? sp->refine_max : 10;
        // the outer residual and corrections live in separate buffers from the
        // inner solver's work vectors
        const size_t colbytes = size_t(n) * C * sizeof(double2);
        if ((st = op_reserve(op, op->d_ref_r, colbytes, "cfie_solve")) ||
            (st = op_reserve(op, op->d_ref_d, colbytes, "cfie_solve")))
            return st;
        double2* R = op->d_ref_r.as<double2>();
        double2* D = op->d_ref_d.as<double2>();
        double2* D2 = nullptr;
        IGB_HIP(hipMemsetAsync(X, 0, n * C * sizeof(double2), s));
        IGB_HIP(hipMemcpyAsync(R, B, n * C * sizeof(double2), hipMemcpyDeviceToDevice, s));
        std::vector<double> bnorm, rnorm;
        if ((st = norms(B, n, C, W.nrm, bnorm, s))) return st;
        rnorm = bnorm;
        res.assign(C, ColumnResult());
        std::vector<char> full(C, 0);   // column refines with the fp64 operator
        for (int c = 0; c < C; ++c) {
            res[c].converged = bnorm[c] == 0.0;
            res[c].relres = res[c].true_rel = res[c].converged ? 0.0 : 1.0;
        }
        for (int outer = 0; outer < refine_max + 3; ++outer) {
            // inner tolerance per column: what the column still needs, at least
            // inner_min on the reduced-precision operator
            std::vector<double> tin(C, 1.0);
            std::vector<int> left(C, 0), left_lo(C, 0), left_hi(C, 0);
            bool any_lo = false, any_hi = false;
            for (int c = 0; c < C; ++c) {
                if (res[c].converged || res[c].iters >= maxit || (!full[c] && outer >= refine_max)) continue;
                left[c] = maxit - res[c].iters;   // maxit bounds the Arnoldi steps over all refinements
                const double need = 0.5 * tol * bnorm[c] / rnorm[c];
                if (full[c]) {
                    tin[c] = need;
                    left_hi[c] = left[c];
                    any_hi = true;
                } else {
                    tin[c] = std::max(inner_min, need);
                    left_lo[c] = left[c];
                    any_lo = true;
                }
            }
            if (!any_lo && !any_hi) break;
            std::vector<ColumnResult> inner(C), part;
            if (any_lo) {
                log.phase = "inner (reduced precision)";
                if ((st = gmres_block(op, W, R, D, left_lo, tin, IGB_PART_ALL | IGB_MV_LOWPREC, s, part, log)))
                    return st;
                for (int c = 0; c < C; ++c)
                    if (left_lo[c]) inner[c] = part[c];
            } else {
                IGB_HIP(hipMemsetAsync(D, 0, n * C * sizeof(double2), s));
            }
            if (any_hi) {
                if (!D2) {
                    if ((st = op_reserve(op, op->d_ref_d2, colbytes, "cfie_solve"))) return st;
                    D2 = op->d_ref_d2.as<double2>();
                }
                log.phase = "inner (fp64)";
                if ((st = gmres_block(op, W, R, D2, left_hi, tin, IGB_PART_ALL, s, part, log))) return st;
                for (int c = 0; c < C; ++c)
                    if (left_hi[c]) inner[c] = part[c];
                hipLaunchKernelGGL(cadd_to, dim3(gb), dim3(256), 0, s, D2, n * C, D);
            }
            hipLaunchKernelGGL(cadd_to, dim3(gb), dim3(256), 0, s, D, n * C, X);
            if ((st = matvec_device(op, reinterpret_cast<const double*>(X), reinterpret_cast<double*>(R), C,
                                    IGB_PART_ALL, s)))
                return st;
            hipLaunchKernelGGL(csub_from_multi, dim3(gb), dim3(256), 0, s, B, n * C, R);
            std::vector<double> rprev = rnorm;
            if ((st = norms(R, n, C, W.nrm, rnorm, s))) return st;
            std::vector<double> undo(C, 0.0);
            bool any_undo = false;
            for (int c = 0; c < C; ++c) {
                if (left[c] == 0) continue;
                res[c].iters += inner[c].iters;
                res[c].applications += inner[c].applications + 1;
                if (!(rnorm[c] < rprev[c])) {
                    // the correction did not reduce the fp64 residual: take it back
                    undo[c] = -1.0;
                    any_undo = true;
                    rnorm[c] = rprev[c];
                    if (full[c]) res[c].iters = maxit;   // no further remedy
                    full[c] = 1;
                } else if (!full[c] && rnorm[c] > ESCALATE * rprev[c]) {
                    full[c] = 1;
                }
                res[c].true_rel = bnorm[c] > 0 ? rnorm[c] / bnorm[c] : 0.0;
                res[c].relres = res[c].true_rel;
                res[c].converged = res[c].true_rel <= tol;
            }
            if (any_undo) {
                // X -= D and R = B - A X for the rejected columns (recomputed for all)
                IGB_HIP(hipMemcpyAsync(W.sc, undo.data(), C * sizeof(double), hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(cscale_multi, dim3(gb), dim3(256), 0, s, D, n, C, W.sc, D);
                hipLaunchKernelGGL(cadd_to, dim3(gb), dim3(256), 0, s, D, n * C, X);
                if ((st = matvec_device(op, reinterpret_cast<const double*>(X), reinterpret_cast<double*>(R), C,
                                        IGB_PART_ALL, s)))
                    return st;
                hipLaunchKernelGGL(csub_from_multi, dim3(gb), dim3(256), 0, s, B, n * C, R);
                IGB_HIP(hipStreamSynchronize(s));
            }
            ++out.refinements;
            if (log.on) {
                int nconv = 0, nesc = 0;
                double worst = 0;
                for (int c = 0; c < C; ++c) {
                    nconv += res[c].converged ? 1 : 0;
                    nesc += full[c] ? 1 : 0;
                    worst = std::max(worst, res[c].true_rel);
                }
                fprintf(stderr, "[igafmm] refinement %d: %d of %d columns converged, %d on fp64, largest true "
                        "relative residual %.2e, %.1f s\n", outer + 1, nconv, C, nesc, worst, log.elapsed());
            }
        }
        for (int c = 0; c < C; ++c) out.escalated += full[c] ? 1 : 0;
    }
    int status = IGB_OK;
    for (int c = 0; c < C; ++c) {
        out.iters = std::max(out.iters, res[c].iters);
        out.matvecs += res[c].applications;
        out.converged += res[c].converged ? 1 : 0;
        out.relres = std::max(out.relres, res[c].relres);
        out.relres_true = std::max(out.relres_true, res[c].true_rel);
        if (!res[c].converged) status = IGB_WARN_NOT_CONVERGED;
    }
    if (info) *info = out;
    return status;
}

}  // namespace igb

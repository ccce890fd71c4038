// Restarted GMRES (Sec. 5.1: GMRES with restart 30 on the CFIE systems) on the
// device.  Arnoldi with classical Gram-Schmidt applied twice (CGS2); all
// vectors stay on the device, only the new Hessenberg column (<= restart+1
// complex numbers) is read back per iteration for the Givens rotations.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <vector>

#include "common.h"

namespace igb {

namespace {

constexpr int RT = 256;

// h[j] (+)= sum_i conj(V[j][i]) w[i]; one workgroup per basis vector, fixed-order tree
__global__ __launch_bounds__(RT) void cdots(const double2* V, int64_t n, const double2* w, double2* h,
                                            int accumulate) {
    __shared__ double2 red[RT];
    const int j = blockIdx.x;
    const double2* v = V + int64_t(j) * n;
    double2 acc = make_double2(0, 0);
    for (int64_t i = threadIdx.x; i < n; i += RT) {
        const double2 a = v[i], b = w[i];
        acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
        acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = RT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[threadIdx.x].x += red[threadIdx.x + s].x;
            red[threadIdx.x].y += red[threadIdx.x + s].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (accumulate) {
            h[j].x += red[0].x;
            h[j].y += red[0].y;
        } else {
            h[j] = red[0];
        }
    }
}

// w[i] -= sum_j c[j] V[j][i]  (c read from device memory)
__global__ void cmaxpy(const double2* V, int nvec, int64_t n, const double2* c, double2* w) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 acc = w[i];
    for (int j = 0; j < nvec; ++j) {
        const double2 a = c[j], v = V[int64_t(j) * n + i];
        acc.x -= a.x * v.x - a.y * v.y;
        acc.y -= a.x * v.y + a.y * v.x;
    }
    w[i] = acc;
}

// out[0] = ||w||_2^2 (single workgroup, fixed order)
__global__ __launch_bounds__(1024) void cnorm2(const double2* w, int64_t n, double* out) {
    __shared__ double red[1024];
    double acc = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) acc = fma(w[i].x, w[i].x, fma(w[i].y, w[i].y, acc));
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void cscale_to(const double2* w, int64_t n, double s, double2* v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) v[i] = make_double2(w[i].x * s, w[i].y * s);
}

// x[i] += sum_j y[j] V[j][i]
__global__ void cupdate(const double2* V, int nvec, int64_t n, const double2* y, double2* x) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 acc = x[i];
    for (int j = 0; j < nvec; ++j) {
        const double2 a = y[j], v = V[int64_t(j) * n + i];
        acc.x += a.x * v.x - a.y * v.y;
        acc.y += a.x * v.y + a.y * v.x;
    }
    x[i] = acc;
}

// r = b - r
__global__ void csub_from(const double2* b, int64_t n, double2* r) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) r[i] = make_double2(b[i].x - r[i].x, b[i].y - r[i].y);
}

using cplx = std::complex<double>;

}  // namespace

namespace {

struct ColumnResult {
    int iters = 0;
    int64_t applications = 0;
    bool converged = false;
    double relres = 1.0;      // recursive estimate at exit
    double true_rel = 1.0;    // ||B - A X|| / ||B|| recomputed with the same operator
};

struct Work {
    int64_t n;
    int m;
    double2 *V, *w, *r, *h, *h2;
    double* nrm;
};

igb_status ensure_work(igb_op op, int m, Work& W) {
    const int64_t n = op->N;
    if (op->krylov_cols < m + 1) {
        op->d_krylov.release();
        op->d_w.release();
        op->d_h.release();
        IGB_HIP(hipMalloc(&op->d_krylov.ptr, size_t(m + 1) * n * sizeof(double2)));
        op->d_krylov.bytes = size_t(m + 1) * n * sizeof(double2);
        IGB_HIP(hipMalloc(&op->d_w.ptr, size_t(4) * n * sizeof(double2)));
        op->d_w.bytes = size_t(4) * n * sizeof(double2);
        IGB_HIP(hipMalloc(&op->d_h.ptr, size_t(2 * (m + 2)) * sizeof(double2) + 64));
        op->d_h.bytes = size_t(2 * (m + 2)) * sizeof(double2) + 64;
        op->dev_bytes += op->d_krylov.bytes + op->d_w.bytes + op->d_h.bytes;
        op->krylov_cols = m + 1;
    }
    W.n = n;
    W.m = m;
    W.V = op->d_krylov.as<double2>();
    W.w = op->d_w.as<double2>();
    W.r = W.w + n;
    W.h = op->d_h.as<double2>();
    W.h2 = W.h + (m + 2);
    W.nrm = reinterpret_cast<double*>(W.h2 + (m + 2));
    return IGB_OK;
}

igb_status norm2(const double2* v, int64_t n, double* dev_tmp, double* out, hipStream_t s) {
    hipLaunchKernelGGL(cnorm2, dim3(1), dim3(1024), 0, s, v, n, dev_tmp);
    IGB_HIP(hipMemcpyAsync(out, dev_tmp, sizeof(double), hipMemcpyDeviceToHost, s));
    IGB_HIP(hipStreamSynchronize(s));
    *out = std::sqrt(*out);
    return IGB_OK;
}

// Restarted GMRES for one column: X = 0 initially, stop at ||B - A X|| <= tol ||B||
// (recursive estimate) or after maxit operator applications.  `mvflags` selects
// the operator (IGB_PART_ALL, optionally with the reduced-precision far field).
igb_status gmres_column(igb_op op, const Work& Wk, const double2* B, double2* X, int maxit, double tol,
                        int mvflags, hipStream_t s, ColumnResult& res) {
    const int64_t n = Wk.n;
    const int m = Wk.m;
    const unsigned gb = unsigned((n + 255) / 256);
    double2 *V = Wk.V, *w = Wk.w, *r = Wk.r, *h = Wk.h, *h2 = Wk.h2;
    double* nrm = Wk.nrm;
    IGB_HIP(hipMemsetAsync(X, 0, n * sizeof(double2), s));
    double bnorm = 0;
    igb_status st;
    if ((st = norm2(B, n, nrm, &bnorm, s))) return st;
    res = ColumnResult();
    res.converged = bnorm == 0.0;
    res.relres = res.true_rel = res.converged ? 0.0 : 1.0;
    IGB_HIP(hipMemcpyAsync(r, B, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
    double rnorm = bnorm;
    std::vector<cplx> H(size_t(m + 1) * m), cs(m), sn(m), g(m + 1);
    std::vector<double2> hh(2 * (m + 1));
    double nrm_h = 0;
    while (!res.converged && res.iters < maxit) {
        hipLaunchKernelGGL(cscale_to, dim3(gb), dim3(256), 0, s, r, n, 1.0 / rnorm, V);
        std::fill(g.begin(), g.end(), cplx(0));
        g[0] = rnorm;
        int j = 0;
        for (; j < m && res.iters < maxit; ++j) {
            if ((st = matvec_device(op, reinterpret_cast<const double*>(V + int64_t(j) * n),
                                    reinterpret_cast<double*>(w), 1, mvflags, s)))
                return st;
            ++res.iters;
            ++res.applications;
            // classical Gram-Schmidt, twice
            hipLaunchKernelGGL(cdots, dim3(j + 1), dim3(RT), 0, s, V, n, w, h, 0);
            hipLaunchKernelGGL(cmaxpy, dim3(gb), dim3(256), 0, s, V, j + 1, n, h, w);
            hipLaunchKernelGGL(cdots, dim3(j + 1), dim3(RT), 0, s, V, n, w, h2, 0);
            hipLaunchKernelGGL(cmaxpy, dim3(gb), dim3(256), 0, s, V, j + 1, n, h2, w);
            hipLaunchKernelGGL(cnorm2, dim3(1), dim3(1024), 0, s, w, n, nrm);
            IGB_HIP(hipGetLastError());
            IGB_HIP(hipMemcpyAsync(hh.data(), h, (j + 1) * sizeof(double2), hipMemcpyDeviceToHost, s));
            IGB_HIP(hipMemcpyAsync(hh.data() + j + 1, h2, (j + 1) * sizeof(double2), hipMemcpyDeviceToHost, s));
            IGB_HIP(hipMemcpyAsync(&nrm_h, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
            IGB_HIP(hipStreamSynchronize(s));
            const double hn = std::sqrt(nrm_h);
            for (int i = 0; i <= j; ++i)
                H[size_t(i) * m + j] = cplx(hh[i].x + hh[j + 1 + i].x, hh[i].y + hh[j + 1 + i].y);
            H[size_t(j + 1) * m + j] = hn;
            if (hn > 0)
                hipLaunchKernelGGL(cscale_to, dim3(gb), dim3(256), 0, s, w, n, 1.0 / hn, V + int64_t(j + 1) * n);
            // Givens rotations
            for (int i = 0; i < j; ++i) {
                cplx a = H[size_t(i) * m + j], bb = H[size_t(i + 1) * m + j];
                H[size_t(i) * m + j] = cs[i] * a + sn[i] * bb;
                H[size_t(i + 1) * m + j] = -std::conj(sn[i]) * a + cs[i] * bb;
            }
            cplx a = H[size_t(j) * m + j], bb = H[size_t(j + 1) * m + j];
            double rr = std::sqrt(std::norm(a) + std::norm(bb));
            if (rr == 0) {
                cs[j] = 1;
                sn[j] = 0;
            } else if (std::abs(a) == 0) {
                cs[j] = 0;
                sn[j] = std::conj(bb) / rr;
            } else {
                cs[j] = std::abs(a) / rr;
                sn[j] = (a / std::abs(a)) * std::conj(bb) / rr;
            }
            H[size_t(j) * m + j] = cs[j] * a + sn[j] * bb;
            H[size_t(j + 1) * m + j] = 0;
            g[j + 1] = -std::conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            res.relres = std::abs(g[j + 1]) / bnorm;
            if (res.relres <= tol || hn == 0) {
                ++j;
                res.converged = true;
                break;
            }
        }
        // y = H^{-1} g (upper triangular j x j), X += V y
        std::vector<cplx> y(j);
        for (int i = j - 1; i >= 0; --i) {
            cplx acc = g[i];
            for (int kk = i + 1; kk < j; ++kk) acc -= H[size_t(i) * m + kk] * y[kk];
            y[i] = acc / H[size_t(i) * m + i];
        }
        std::vector<double2> yd(j);
        for (int i = 0; i < j; ++i) yd[i] = make_double2(y[i].real(), y[i].imag());
        IGB_HIP(hipMemcpyAsync(h, yd.data(), j * sizeof(double2), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(cupdate, dim3(gb), dim3(256), 0, s, V, j, n, h, X);
        // residual of the same operator: r = B - A X
        if ((st = matvec_device(op, reinterpret_cast<const double*>(X), reinterpret_cast<double*>(r), 1, mvflags, s)))
            return st;
        ++res.applications;
        hipLaunchKernelGGL(csub_from, dim3(gb), dim3(256), 0, s, B, n, r);
        IGB_HIP(hipGetLastError());
        if ((st = norm2(r, n, nrm, &rnorm, s))) return st;
        res.true_rel = bnorm > 0 ? rnorm / bnorm : 0.0;
    }
    return IGB_OK;
}

__global__ void cadd_to(const double2* d, int64_t n, double2* x) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = make_double2(x[i].x + d[i].x, x[i].y + d[i].y);
}

}  // namespace

igb_status gmres_device(igb_op op, const double* b_in, double* x_out, int ndir, const igb_solve_params* sp,
                        igb_solve_info* info, hipStream_t s) {
    const int64_t n = op->N;
    const int m = sp->restart > 0 ? sp->restart : 30;
    const int maxit = sp->maxit > 0 ? sp->maxit : 1000;
    const double tol = sp->tol > 0 ? sp->tol : 1e-8;
    const bool mixed = op->prm.precision != IGB_FP64;
    Work W;
    igb_status st;
    if ((st = ensure_work(op, m, W))) return st;
    const unsigned gb = unsigned((n + 255) / 256);
    igb_solve_info out{};
    int status = IGB_OK;
    for (int col = 0; col < ndir; ++col) {
        const double2* B = reinterpret_cast<const double2*>(b_in) + int64_t(col) * n;
        double2* X = reinterpret_cast<double2*>(x_out) + int64_t(col) * n;
        ColumnResult res;
        if (!mixed) {
            if ((st = gmres_column(op, W, B, X, maxit, tol, IGB_PART_ALL, s, res))) return st;
        } else {
            // iterative refinement: inner GMRES on the reduced-precision far field,
            // outer residual with the fp64 operator
            double2* R = W.w + 2 * n;   // outer residual
            double2* D = W.w + 3 * n;   // correction
            const double inner_min = sp->inner_tol > 0 ? sp->inner_tol
                                     : (op->prm.precision == IGB_MIX_FP32 ? 0.0 : 1e-3);
            const int refine_max = sp->refine_max > 0 ? sp->refine_max : 10;
            IGB_HIP(hipMemsetAsync(X, 0, n * sizeof(double2), s));
            IGB_HIP(hipMemcpyAsync(R, B, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
            double bnorm = 0, rnorm = 0;
            if ((st = norm2(B, n, W.nrm, &bnorm, s))) return st;
            rnorm = bnorm;
            ColumnResult acc;
            acc.converged = bnorm == 0.0;
            acc.true_rel = acc.converged ? 0.0 : 1.0;
            for (int outer = 0; outer < refine_max && !acc.converged && acc.iters < maxit; ++outer) {
                const double tin = std::max(inner_min, 0.5 * tol * bnorm / rnorm);
                ColumnResult inner;
                if ((st = gmres_column(op, W, R, D, maxit - acc.iters, tin, IGB_PART_ALL | IGB_MV_LOWPREC, s, inner)))
                    return st;
                acc.iters += inner.iters;
                acc.applications += inner.applications;
                hipLaunchKernelGGL(cadd_to, dim3(gb), dim3(256), 0, s, D, n, X);
                if ((st = matvec_device(op, reinterpret_cast<const double*>(X), reinterpret_cast<double*>(R), 1,
                                        IGB_PART_ALL, s)))
                    return st;
                ++acc.applications;
                hipLaunchKernelGGL(csub_from, dim3(gb), dim3(256), 0, s, B, n, R);
                if ((st = norm2(R, n, W.nrm, &rnorm, s))) return st;
                acc.true_rel = bnorm > 0 ? rnorm / bnorm : 0.0;
                acc.relres = acc.true_rel;
                acc.converged = acc.true_rel <= tol;
                ++out.refinements;
            }
            res = acc;
        }
        out.iters = std::max(out.iters, res.iters);
        out.matvecs += res.applications;
        out.converged += res.converged ? 1 : 0;
        out.relres = std::max(out.relres, res.relres);
        out.relres_true = std::max(out.relres_true, res.true_rel);
        if (!res.converged) status = IGB_WARN_NOT_CONVERGED;
    }
    if (info) *info = out;
    return status;
}

}  // namespace igb

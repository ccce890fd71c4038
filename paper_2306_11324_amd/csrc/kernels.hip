// Device side of the igafmm library (gfx950): near-field quadrature, coupling
// assembly, the H^2 matrix-vector pipeline, right-hand sides and far field.
// All floating point is fp64; complex values are double2 (re, im).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "common.h"

namespace igb {

// --------------------------------------------------------------------------
// small device helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// c + a * b
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// Bernstein polynomials of degree p <= 3 on [0,1] and their derivatives
__device__ __forceinline__ void bernstein(int p, double s, double* b, double* db) {
    const double t = 1.0 - s;
    if (p == 0) {
        b[0] = 1; db[0] = 0;
    } else if (p == 1) {
        b[0] = t; b[1] = s; db[0] = -1; db[1] = 1;
    } else if (p == 2) {
        b[0] = t * t; b[1] = 2 * s * t; b[2] = s * s;
        db[0] = -2 * t; db[1] = 2 * (t - s); db[2] = 2 * s;
    } else {
        b[0] = t * t * t; b[1] = 3 * s * t * t; b[2] = 3 * s * s * t; b[3] = s * s * s;
        db[0] = -3 * t * t; db[1] = 3 * t * t - 6 * s * t; db[2] = 6 * s * t - 3 * s * s; db[3] = 3 * s * s;
    }
}

struct GeoPt {
    double x[3];   // F
    double fs[3];  // dF/ds (element-local)
    double ft[3];  // dF/dt
};

// rational Bezier element map at local (s, t)
__device__ __forceinline__ void eval_geo(const double* __restrict__ bez, int pu, int pv, double s,
                                         double t, GeoPt& g) {
    double bu[4], dbu[4], bv[4], dbv[4];
    bernstein(pu, s, bu, dbu);
    bernstein(pv, t, bv, dbv);
    double P[4] = {0, 0, 0, 0}, Ps[4] = {0, 0, 0, 0}, Pt[4] = {0, 0, 0, 0};
    for (int j = 0; j <= pv; ++j) {
        double rP[4] = {0, 0, 0, 0}, rPs[4] = {0, 0, 0, 0};
        for (int i = 0; i <= pu; ++i) {
            const double* H = bez + (j * (PGMAX + 1) + i) * 4;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                rP[c] = fma(bu[i], H[c], rP[c]);
                rPs[c] = fma(dbu[i], H[c], rPs[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            P[c] = fma(bv[j], rP[c], P[c]);
            Ps[c] = fma(bv[j], rPs[c], Ps[c]);
            Pt[c] = fma(dbv[j], rP[c], Pt[c]);
        }
    }
    const double iw = 1.0 / P[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        g.x[c] = P[c] * iw;
        g.fs[c] = (Ps[c] - g.x[c] * Ps[3]) * iw;
        g.ft[c] = (Pt[c] - g.x[c] * Pt[3]) * iw;
    }
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// local B-splines b_{ex+a}(s), a = 0..p, from the element's extraction rows
template <int P>
__device__ __forceinline__ void eval_basis1(const double* __restrict__ C, double s, double* phi, double* dphi) {
    double b[4], db[4];
    bernstein(P, s, b, db);
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        double v = 0, d = 0;
#pragma unroll
        for (int k = 0; k <= P; ++k) {
            v = fma(C[a * (P + 1) + k], b[k], v);
            d = fma(C[a * (P + 1) + k], db[k], d);
        }
        phi[a] = v;
        if (dphi) dphi[a] = d;
    }
}

__device__ __forceinline__ void d4_apply(int code, double s, double t, double& a, double& b) {
    a = s;
    b = t;
    if (code & 4) {
        double x = a;
        a = b;
        b = x;
    }
    if (code & 1) a = 1.0 - a;
    if (code & 2) b = 1.0 - b;
}

struct ElemRef {
    const double* bez;
    int pu, pv, ex, ey;
};

__device__ __forceinline__ ElemRef elem_ref(const double* bez, const int* pg, int nel1, int64_t e) {
    ElemRef r;
    r.bez = bez + e * NBZ * 4;
    r.pu = pg[2 * e];
    r.pv = pg[2 * e + 1];
    int64_t rem = e % (int64_t(nel1) * nel1);
    r.ey = int(rem / nel1);
    r.ex = int(rem % nel1);
    return r;
}

// The pulled-back kernel of the sound-soft family  ck a_y H (x-y).n~_x + cv a_x a_y G
// with G = e^{i kappa r}/(4 pi r), H = G (i kappa r - 1)/r^2 (Sec. 4.2, eq. of
// the pulled-back kernel, applied to K* and V): ck = 1, cv = -i eta for the
// CFIE of the D2N system, cv = 1 (V alone) or ck = 1, cv = 0 (K* alone) for the
// single-layer formulations.
__device__ __forceinline__ double2 kernel_soft(const double* X, const double* NX, double ax,
                                               const double* Y, double ay, double kappa, SoftMix mix) {
    const double d0 = X[0] - Y[0], d1 = X[1] - Y[1], d2 = X[2] - Y[2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const double r = sqrt(r2);
    const double ir = 1.0 / r;
    const double kr = kappa * r;
    double sn, cs;
    sincos(kr, &sn, &cs);
    const double dn = d0 * NX[0] + d1 * NX[1] + d2 * NX[2];
    const double c4 = 0.07957747154594767 * ir;        // 1/(4 pi r)
    const double h = mix.ck * ay * dn * ir * ir * c4;   // ck a_y (x-y).n~_x / (4 pi r^3)
    const double v = ax * ay * c4;
    return make_double2(h * (-cs - sn * kr) + v * (mix.cv.x * cs - mix.cv.y * sn),
                        h * (cs * kr - sn) + v * (mix.cv.x * sn + mix.cv.y * cs));
}

// --------------------------------------------------------------------------
// Near field: regular element pairs (tensor Gauss of order n on both elements)
// --------------------------------------------------------------------------
constexpr int NEAR_THREADS = 256;
constexpr int NGMAX = 16;

struct NearArgs {
    const double* bez;
    const int* pg;
    const double* C1;
    const double* gl;        // [NGMAX+1][2][NGMAX]: Gauss nodes / weights on [0,1] per order
    const int* pair_e;       // near pair -> target element
    const int* pair_f;       // near pair -> source element
    const int* pair_kind;
    const int* list;         // near pairs handled by this launch
    int64_t nlist;
    int64_t slot0;           // staging slot = pair - slot0
    double2* stage;          // [slots][nloc*nloc]
    int nel1;
    double kappa, eta;       // eta: coupling of the sound-hard CFIE
    SoftMix mix;             // kernel of the sound-soft family
    HardMix hmix;            // kernel of the sound-hard family
    double2 cm;              // multiple of the mass matrix added on identical pairs
    // singular rules: per class (0 vertex, 1 edge, 2 identical) points (s1,s2,r1,r2,w)
    const double* rule[3];
    int rule_n[3];
    int mass_order;
};

// Kernel values at one point pair (element-local coordinates, n~ unnormalised):
//   soft: s = ck a_y H (x-y).n~_x + cv a_x a_y G                      (ck K* + cv V)
//   hard: s = ck a_x H (y-x).n~_y - cw kappa^2 G n~_x.n~_y            (ck K, kappa^2 part of cw W)
//         g = cw G, multiplying the curl product c_i(x).c_j(y)         (curl part of cw W)
//         (the CFIE: ck = -1, cw = -i eta)
struct KVal {
    double2 s, g;
};

template <bool HARD>
__device__ __forceinline__ KVal kernel_pair(const double* X, const double* NX, double ax, const double* Y,
                                            const double* NY, double ay, double kappa, SoftMix mix, HardMix hmix) {
    KVal k;
    if (!HARD) {
        k.s = kernel_soft(X, NX, ax, Y, ay, kappa, mix);
        k.g = make_double2(0, 0);
        return k;
    }
    const double d0 = X[0] - Y[0], d1 = X[1] - Y[1], d2 = X[2] - Y[2];
    const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double ir = 1.0 / r;
    const double kr = kappa * r;
    double sn, cs;
    sincos(kr, &sn, &cs);
    const double c4 = 0.07957747154594767 * ir;
    const double dny = d0 * NY[0] + d1 * NY[1] + d2 * NY[2];
    const double nn = NX[0] * NY[0] + NX[1] * NY[1] + NX[2] * NY[2];
    // K kernel a_x H (y-x).n~_y = kn (cs + i sn) (i kr - 1), kn = -a_x (x-y).n~_y / (4 pi r^3)
    const double kn = -ax * dny * ir * ir * c4;
    const double2 kk = make_double2(kn * (-cs - sn * kr), kn * (cs * kr - sn));
    const double v = -kappa * kappa * nn * c4;   // W's kappa^2 part: v (cs + i sn)
    const double2 w = make_double2(v * cs, v * sn);
    const double2 g = make_double2(c4 * cs, c4 * sn);
    k.s = cadd(cmul(hmix.ck, kk), cmul(hmix.cw, w));
    k.g = cmul(hmix.cw, g);
    return k;
}

// Point data of one element at local (s,t): position, n~, a and, per local basis
// function, w*phi (component 0) and for the hypersingular part w*c with
// c = d_s phi F_t - d_t phi F_s (components 1..3).
template <int P, bool HARD>
__device__ __forceinline__ void point_data(const ElemRef& R, const double* Cu, const double* Cv, double s,
                                           double t, double w, double* g7, double* ph /*[NL][NV]*/) {
    constexpr int NV = HARD ? 4 : 1;
    GeoPt G;
    eval_geo(R.bez, R.pu, R.pv, s, t, G);
    double nt[3];
    cross3(G.fs, G.ft, nt);
    g7[0] = G.x[0]; g7[1] = G.x[1]; g7[2] = G.x[2];
    g7[3] = nt[0]; g7[4] = nt[1]; g7[5] = nt[2];
    g7[6] = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
    double bu[P + 1], bv[P + 1], dbu[P + 1], dbv[P + 1];
    eval_basis1<P>(Cu, s, bu, dbu);
    eval_basis1<P>(Cv, t, bv, dbv);
#pragma unroll
    for (int av = 0; av <= P; ++av)
#pragma unroll
        for (int au = 0; au <= P; ++au) {
            double* o = ph + (av * (P + 1) + au) * NV;
            o[0] = w * bv[av] * bu[au];
            if (HARD) {
                const double ds = bv[av] * dbu[au], dt = dbv[av] * bu[au];
#pragma unroll
                for (int c = 0; c < 3; ++c) o[1 + c] = w * (ds * G.ft[c] - dt * G.fs[c]);
            }
        }
}

// --------------------------------------------------------------------------
// Near field: regular element pairs, tensor Gauss rules of orders (nu, nv) on
// each element (nu * nv <= MAXQ points; the orders may differ between the two
// elements and between directions).  Kernel values are produced in chunks of
// CI test points in LDS; thread items (j, a) accumulate
// T[j][a] = sum_i w phi_a(x_i) k(x_i, y_j); finally B[a][b] = sum_j T[j][a] . w phi_b(y_j).
// --------------------------------------------------------------------------
template <int P, bool HARD, int MAXQ>
__global__ __launch_bounds__(NEAR_THREADS) void near_regular(NearArgs A) {
    constexpr int NL = (P + 1) * (P + 1);
    constexpr int NV = HARD ? 4 : 1;
    constexpr int NK = HARD ? 2 : 1;
    constexpr int CI = 8;
    constexpr int BUF = (CI * MAXQ * NK > MAXQ * NL) ? CI * MAXQ * NK : MAXQ * NL;
    constexpr int ITEMS = (MAXQ * NL + NEAR_THREADS - 1) / NEAR_THREADS;
    __shared__ double xg[MAXQ][7];
    __shared__ double yg[MAXQ][7];
    __shared__ double px[MAXQ][NL * NV];
    __shared__ double py[MAXQ][NL * NV];
    __shared__ double2 buf[BUF];

    const int64_t item = blockIdx.x;
    if (item >= A.nlist) return;
    const int k = A.list[item];
    const int e = A.pair_e[k], f = A.pair_f[k];
    const int kind = A.pair_kind[k];
    const int nxu = (kind >> 8) & 15, nxv = (kind >> 12) & 15, nyu = (kind >> 16) & 15, nyv = (kind >> 20) & 15;
    const int nx = nxu * nxv, ny = nyu * nyv;
    const int tid = threadIdx.x;

    if (tid < nx + ny) {
        const bool isx = tid < nx;
        const int i = isx ? tid : tid - nx;
        const int nu = isx ? nxu : nyu, nv = isx ? nxv : nyv;
        const double* gu = A.gl + nu * 2 * NGMAX;
        const double* gv = A.gl + nv * 2 * NGMAX;
        const ElemRef R = elem_ref(A.bez, A.pg, A.nel1, isx ? e : f);
        point_data<P, HARD>(R, A.C1 + R.ex * (P + 1) * (P + 1), A.C1 + R.ey * (P + 1) * (P + 1), gu[i % nu],
                            gv[i / nu], gu[NGMAX + i % nu] * gv[NGMAX + i / nu], isx ? xg[i] : yg[i],
                            isx ? px[i] : py[i]);
    }
    __syncthreads();

    double2 acc[ITEMS][NV];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[it][v] = make_double2(0, 0);
    for (int i0 = 0; i0 < nx; i0 += CI) {
        const int ci = min(CI, nx - i0);
        for (int idx = tid; idx < ci * ny; idx += NEAR_THREADS) {
            const int i = i0 + idx / ny, j = idx % ny;
            const KVal kv = kernel_pair<HARD>(xg[i], xg[i] + 3, xg[i][6], yg[j], yg[j] + 3, yg[j][6], A.kappa, A.mix,
                                                 A.hmix);
            buf[idx * NK] = kv.s;
            if (HARD) buf[idx * NK + 1] = kv.g;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int w = tid + it * NEAR_THREADS;
            if (w < ny * NL) {
                const int j = w / NL, a = w % NL;
                for (int ii = 0; ii < ci; ++ii) {
                    const double* pxv = &px[i0 + ii][a * NV];
                    const double2 ks = buf[(ii * ny + j) * NK];
                    acc[it][0].x = fma(pxv[0], ks.x, acc[it][0].x);
                    acc[it][0].y = fma(pxv[0], ks.y, acc[it][0].y);
                    if (HARD) {
                        const double2 kg = buf[(ii * ny + j) * NK + 1];
#pragma unroll
                        for (int v = 1; v < NV; ++v) {
                            acc[it][v].x = fma(pxv[v], kg.x, acc[it][v].x);
                            acc[it][v].y = fma(pxv[v], kg.y, acc[it][v].y);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    // one component v at a time: T[j][a] into LDS, then B[a][b] += sum_j T[j][a] py[j][b][v]
    // (keeps the buffer at MAXQ * NL entries, which the degree-3 hypersingular case needs)
    const int a = tid / NL, b = tid % NL;
    double2 sum = make_double2(0, 0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const int w = tid + it * NEAR_THREADS;
            if (w < ny * NL) buf[w] = acc[it][v];
        }
        __syncthreads();
        if (tid < NL * NL)
            for (int j = 0; j < ny; ++j) {
                const double2 t = buf[j * NL + a];
                const double y = py[j][b * NV + v];
                sum.x = fma(t.x, y, sum.x);
                sum.y = fma(t.y, y, sum.y);
            }
        __syncthreads();
    }
    if (tid < NL * NL) A.stage[(int64_t(k) - A.slot0) * NL * NL + tid] = sum;
}

// --------------------------------------------------------------------------
// Near field: touching element pairs (Duffy-type rules on [0,1]^4), points in
// batches staged through LDS; output (a,b) accumulated by SPLIT threads each.
// --------------------------------------------------------------------------
template <int P, bool HARD>
__global__ __launch_bounds__(NEAR_THREADS) void near_singular(NearArgs A) {
    constexpr int NL = (P + 1) * (P + 1);
    constexpr int NV = HARD ? 4 : 1;
    constexpr int BATCH = HARD ? 64 : NEAR_THREADS;
    constexpr int SPLIT = NEAR_THREADS / (NL * NL) > 0 ? NEAR_THREADS / (NL * NL) : 1;
    __shared__ KVal kq[BATCH];
    __shared__ double px[BATCH][NL * NV];
    __shared__ double py[BATCH][NL * NV];
    __shared__ double2 red[NEAR_THREADS];

    const int64_t item = blockIdx.x;
    if (item >= A.nlist) return;
    const int k = A.list[item];
    const int e = A.pair_e[k], f = A.pair_f[k];
    const int kind = A.pair_kind[k];
    const int cls = kind & 15;
    const int te = (kind >> 16) & 7, tf = (kind >> 20) & 7;
    const int ri = cls == 4 ? 2 : cls == 2 ? 1 : 0;
    const double* rule = A.rule[ri];
    const int Q = A.rule_n[ri];
    const int tid = threadIdx.x;
    const ElemRef Re = elem_ref(A.bez, A.pg, A.nel1, e);
    const ElemRef Rf = elem_ref(A.bez, A.pg, A.nel1, f);
    const double* Ce_u = A.C1 + Re.ex * (P + 1) * (P + 1);
    const double* Ce_v = A.C1 + Re.ey * (P + 1) * (P + 1);
    const double* Cf_u = A.C1 + Rf.ex * (P + 1) * (P + 1);
    const double* Cf_v = A.C1 + Rf.ey * (P + 1) * (P + 1);

    const int out = tid % (NL * NL), part = tid / (NL * NL);
    const int oa = out / NL, ob = out % NL;
    double2 acc = make_double2(0, 0);
    for (int base = 0; base < Q; base += BATCH) {
        if (tid < BATCH) {
            const int qi = base + tid;
            if (qi < Q) {
                const double* r = rule + int64_t(qi) * 5;
                double s, t, u, v;
                d4_apply(te, r[0], r[1], s, t);
                d4_apply(tf, r[2], r[3], u, v);
                double gxv[7], gyv[7];
                point_data<P, HARD>(Re, Ce_u, Ce_v, s, t, 1.0, gxv, px[tid]);
                point_data<P, HARD>(Rf, Cf_u, Cf_v, u, v, 1.0, gyv, py[tid]);
                KVal kv = kernel_pair<HARD>(gxv, gxv + 3, gxv[6], gyv, gyv + 3, gyv[6], A.kappa, A.mix, A.hmix);
                kv.s = cscale(kv.s, r[4]);
                kv.g = cscale(kv.g, r[4]);
                kq[tid] = kv;
            } else {
                kq[tid].s = make_double2(0, 0);
                kq[tid].g = make_double2(0, 0);
#pragma unroll
                for (int a = 0; a < NL * NV; ++a) {
                    px[tid][a] = 0;
                    py[tid][a] = 0;
                }
            }
        }
        __syncthreads();
        if (part < SPLIT) {
            for (int q = part; q < BATCH; q += SPLIT) {
                const double w = px[q][oa * NV] * py[q][ob * NV];
                acc.x = fma(w, kq[q].s.x, acc.x);
                acc.y = fma(w, kq[q].s.y, acc.y);
                if (HARD) {
                    double c = 0;
#pragma unroll
                    for (int v = 1; v < NV; ++v) c = fma(px[q][oa * NV + v], py[q][ob * NV + v], c);
                    acc.x = fma(c, kq[q].g.x, acc.x);
                    acc.y = fma(c, kq[q].g.y, acc.y);
                }
            }
        }
        __syncthreads();
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < NL * NL) {
        double2 sum = make_double2(0, 0);
        for (int g2 = 0; g2 < SPLIT; ++g2) sum = cadd(sum, red[g2 * NL * NL + tid]);
        if (cls == 4 && (A.cm.x != 0 || A.cm.y != 0)) {
            // + cm times the mass matrix on the identical pair: int phi_a phi_b a
            const int n = A.mass_order;
            const double* gx = A.gl + n * 2 * NGMAX;
            const double* gw = gx + NGMAX;
            double m = 0;
            for (int i = 0; i < n * n; ++i) {
                const double ss = gx[i % n], tt = gx[i / n];
                GeoPt G;
                eval_geo(Re.bez, Re.pu, Re.pv, ss, tt, G);
                double nt[3];
                cross3(G.fs, G.ft, nt);
                double bu[P + 1], bv[P + 1];
                eval_basis1<P>(Ce_u, ss, bu, nullptr);
                eval_basis1<P>(Ce_v, tt, bv, nullptr);
                const double pa = bv[oa / (P + 1)] * bu[oa % (P + 1)];
                const double pb = bv[ob / (P + 1)] * bu[ob % (P + 1)];
                m += gw[i % n] * gw[i / n] * sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]) * pa * pb;
            }
            sum.x += A.cm.x * m;
            sum.y += A.cm.y * m;
        }
        A.stage[(int64_t(k) - A.slot0) * NL * NL + tid] = sum;
    }
}

// --------------------------------------------------------------------------
// Near field: deterministic gather of the staged element blocks into the CSR
// values of the solution space.  One workgroup per row; each nonzero sums its
// contributions in a fixed order (representatives, elements, source elements).
// --------------------------------------------------------------------------
struct CsrArgs {
    const int64_t* row_ptr;
    const int* col;
    double2* val;
    const int64_t* near_ptr;
    const int* near_src;
    const double2* stage;
    int64_t slot0;
    int64_t e_lo, e_hi;          // target elements whose pairs are staged
    const int* s0_ptr;           // null for S^2 (soft)
    const int* s0_reps;
    int64_t row0;
    int nel1, k;
};

template <int P>
__global__ void near_gather_csr(CsrArgs A) {
    constexpr int NL = (P + 1) * (P + 1);
    const int64_t row = A.row0 + blockIdx.x;
    const int64_t beg = A.row_ptr[row], end = A.row_ptr[row + 1];
    const int64_t kk = int64_t(A.k) * A.k;
    const int r0 = A.s0_ptr ? A.s0_ptr[row] : int(row);
    const int r1 = A.s0_ptr ? A.s0_ptr[row + 1] : int(row) + 1;
    for (int64_t idx = beg + threadIdx.x; idx < end; idx += blockDim.x) {
        const int colv = A.col[idx];
        const int c0 = A.s0_ptr ? A.s0_ptr[colv] : colv;
        const int c1 = A.s0_ptr ? A.s0_ptr[colv + 1] : colv + 1;
        double2 acc = make_double2(0, 0);
        for (int ri = r0; ri < r1; ++ri) {
            const int64_t i = A.s0_ptr ? A.s0_reps[ri] : ri;
            const int pj = int(i / kk), rem = int(i % kk), iv = rem / A.k, iu = rem % A.k;
            for (int ey = max(0, iv - P); ey <= min(iv, A.nel1 - 1); ++ey)
                for (int ex = max(0, iu - P); ex <= min(iu, A.nel1 - 1); ++ex) {
                    const int64_t e = (int64_t(pj) * A.nel1 + ey) * A.nel1 + ex;
                    if (e < A.e_lo || e >= A.e_hi) continue;
                    const int a = (iv - ey) * (P + 1) + (iu - ex);
                    const int64_t nb = A.near_ptr[e], ne = A.near_ptr[e + 1];
                    for (int ci = c0; ci < c1; ++ci) {
                        const int64_t j = A.s0_ptr ? A.s0_reps[ci] : ci;
                        const int qj = int(j / kk), rj = int(j % kk), jv = rj / A.k, ju = rj % A.k;
                        for (int fy = max(0, jv - P); fy <= min(jv, A.nel1 - 1); ++fy)
                            for (int fx = max(0, ju - P); fx <= min(ju, A.nel1 - 1); ++fx) {
                                const int f = int((int64_t(qj) * A.nel1 + fy) * A.nel1 + fx);
                                int64_t lo = nb, hi = ne;
                                while (lo < hi) {
                                    int64_t mid = (lo + hi) >> 1;
                                    if (A.near_src[mid] < f) lo = mid + 1;
                                    else hi = mid;
                                }
                                if (lo < ne && A.near_src[lo] == f) {
                                    const int b = (jv - fy) * (P + 1) + (ju - fx);
                                    acc = cadd(acc, A.stage[(lo - A.slot0) * NL * NL + a * NL + b]);
                                }
                            }
                    }
                }
        }
        A.val[idx] = cadd(A.val[idx], acc);
    }
}

// --------------------------------------------------------------------------
// Far field: node geometry and coupling matrices
// --------------------------------------------------------------------------
// Per cluster and Chebyshev node: x(3), n~(3), a, 0, F_u(3), F_v(3), 0, 0 with
// derivatives w.r.t. the patch parameters.
__global__ void node_geometry(const double* bez, const int* pg, int nel1, int npatch, int L,
                              const int64_t* clu_off, const double* tnodes, int q, double* nodes) {
    const int nq = (q + 1) * (q + 1);
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t total = clu_off[L + 1] * nq;
    if (gid >= total) return;
    const int64_t c = gid / nq;
    const int a = int(gid % nq);
    int l = 0;
    while (clu_off[l + 1] <= c) ++l;
    const int64_t loc = c - clu_off[l];
    const int n = 1 << l;
    const int patch = int(loc / (int64_t(n) * n));
    const int rem = int(loc % (int64_t(n) * n));
    const int cy = rem / n, cx = rem % n;
    const double u = (cx + tnodes[a % (q + 1)]) / n, v = (cy + tnodes[a / (q + 1)]) / n;
    const int ex = min(int(u * nel1), nel1 - 1), ey = min(int(v * nel1), nel1 - 1);
    const int64_t e = (int64_t(patch) * nel1 + ey) * nel1 + ex;
    GeoPt G;
    eval_geo(bez + e * NBZ * 4, pg[2 * e], pg[2 * e + 1], u * nel1 - ex, v * nel1 - ey, G);
    double fu[3], fv[3], nt[3];
    for (int i = 0; i < 3; ++i) {
        fu[i] = G.fs[i] * nel1;
        fv[i] = G.ft[i] * nel1;
    }
    cross3(fu, fv, nt);
    double* o = nodes + gid * 16;
    o[0] = G.x[0]; o[1] = G.x[1]; o[2] = G.x[2];
    o[3] = nt[0]; o[4] = nt[1]; o[5] = nt[2];
    o[6] = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
    o[7] = 0;
    o[8] = fu[0]; o[9] = fu[1]; o[10] = fu[2];
    o[11] = fv[0]; o[12] = fv[1]; o[13] = fv[2];
    o[14] = 0; o[15] = 0;
}

// coupling[pair][b*nq + a] = k(x_a of target, y_b of source)
__global__ void coupling_soft(const double* nodes, const int* pair_tgt, const int* pair_src,
                              int64_t npairs, int nq, double kappa, SoftMix mix, double2* coup) {
    for (int64_t pr = blockIdx.x; pr < npairs; pr += gridDim.x) {
        const double* T = nodes + int64_t(pair_tgt[pr]) * nq * 16;
        const double* S = nodes + int64_t(pair_src[pr]) * nq * 16;
        double2* out = coup + pr * nq * nq;
        for (int idx = threadIdx.x; idx < nq * nq; idx += blockDim.x) {
            const int b = idx / nq, a = idx % nq;
            const double* X = T + a * 16;
            const double* Y = S + b * 16;
            out[idx] = kernel_soft(X, X + 3, X[6], Y, Y[6], kappa, mix);
        }
    }
}

// sound-hard raw kernels at a node pair: G = e^{i kappa r}/(4 pi r) and
// H = G (i kappa r - 1)/r^2 (so grad_y G = H (y - x))
__device__ __forceinline__ void kernel_gh(const double* X, const double* Y, double kappa, double2& G, double2& H) {
    const double d0 = X[0] - Y[0], d1 = X[1] - Y[1], d2 = X[2] - Y[2];
    const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double ir = 1.0 / r, kr = kappa * r;
    double sn, cs;
    sincos(kr, &sn, &cs);
    const double c4 = 0.07957747154594767 * ir;
    G = make_double2(c4 * cs, c4 * sn);
    H = make_double2(c4 * ir * ir * (-cs - sn * kr), c4 * ir * ir * (cs * kr - sn));
}

// sound-hard: raw kernels at node pairs, two tiles per pair, G[b*nq + a] then
// H[b*nq + a]; the node-wise factors (measures, normals, tangents) are applied
// around the coupling product
__global__ void coupling_hard(const double* nodes, const int* pair_tgt, const int* pair_src, int64_t npairs,
                              int nq, double kappa, double2* coup) {
    for (int64_t pr = blockIdx.x; pr < npairs; pr += gridDim.x) {
        const double* T = nodes + int64_t(pair_tgt[pr]) * nq * 16;
        const double* S = nodes + int64_t(pair_src[pr]) * nq * 16;
        double2* out = coup + pr * nq * nq * 2;
        for (int idx = threadIdx.x; idx < nq * nq; idx += blockDim.x) {
            const int b = idx / nq, a = idx % nq;
            kernel_gh(T + a * 16, S + b * 16, kappa, out[idx], out[nq * nq + idx]);
        }
    }
}

// --------------------------------------------------------------------------
// H^2 matrix-vector pipeline
// --------------------------------------------------------------------------
// Multi-column layouts (ncol columns C):  vectors [C][n]; moments
// [kind][cluster][nq][C]; M2L partials [chunk][nvec][nq][C]; leaf buffers
// [kind][leaf][C][w*w].  Every kernel computes each column with the same
// operation order whatever ncol is, so a column's result does not depend on
// the batch it is computed in.

// x2[r][i] = x0[r][s2_to_s0[i]]  (S^0 -> S^2 injection)
__global__ void glue_gather(const int* s2_to_s0, const double2* x0, int64_t n0, double2* x2, int64_t n2, int ncol) {
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= n2 * ncol) return;
    const int64_t r = gid / n2, i = gid % n2;
    x2[gid] = x0[r * n0 + s2_to_s0[i]];
}

// leaf moments  xh[leaf][a][r] = sum_{window} m_v[cy][av][iv] m_u[cx][au][iu] x[r][patch][iv][iu]
// leaf_moments with one workgroup per (leaf, column): the leaf's B-spline
// window and moment tables in LDS, sum-factorised (rows over u, then v) in the
// same order as leaf_moments, for windows of at most LM_W coefficients per side.
constexpr int LM_W = 20;
__global__ __launch_bounds__(64) void leaf_moments_wg(const double2* __restrict__ x, int64_t xstride,
                                                      const double* __restrict__ m1, int q, int d, int p, int L,
                                                      int k, int64_t leaf_off, double2* __restrict__ xh,
                                                      int deriv_u, int deriv_v, int64_t m1_stride_kind, int ncol) {
    __shared__ double2 X[LM_W * LM_W];
    __shared__ double2 tmp[LM_W * (QMAX + 1)];
    __shared__ double mu[(QMAX + 1) * LM_W], mv[(QMAX + 1) * LM_W];
    const int q1 = q + 1, nq = q1 * q1, tid = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int r = blockIdx.y;
    const int n = 1 << L, s = 1 << d, w = s + p;
    const int patch = int(c / (int64_t(n) * n));
    const int rem = int(c % (int64_t(n) * n));
    const int cy = rem / n, cx = rem % n;
    const double2* Xg = x + r * xstride + int64_t(patch) * k * k + int64_t(cy) * s * k + int64_t(cx) * s;
    for (int i = tid; i < w * w; i += 64) X[i] = Xg[int64_t(i / w) * k + i % w];
    for (int i = tid; i < q1 * w; i += 64) {
        mu[i] = m1[deriv_u * m1_stride_kind + int64_t(cx) * q1 * w + i];
        mv[i] = m1[deriv_v * m1_stride_kind + int64_t(cy) * q1 * w + i];
    }
    __syncthreads();
    for (int i = tid; i < w * q1; i += 64) {
        const int iv = i / q1, au = i % q1;
        double2 row = make_double2(0, 0);
        for (int iu = 0; iu < w; ++iu) {
            const double2 xv = X[iv * w + iu];
            row.x = fma(mu[au * w + iu], xv.x, row.x);
            row.y = fma(mu[au * w + iu], xv.y, row.y);
        }
        tmp[i] = row;
    }
    __syncthreads();
    for (int a = tid; a < nq; a += 64) {
        const int au = a % q1, av = a / q1;
        double2 acc = make_double2(0, 0);
        for (int iv = 0; iv < w; ++iv) {
            const double2 row = tmp[iv * q1 + au];
            acc.x = fma(mv[av * w + iv], row.x, acc.x);
            acc.y = fma(mv[av * w + iv], row.y, acc.y);
        }
        xh[((leaf_off + c) * nq + a) * ncol + r] = acc;
    }
}

__global__ void leaf_moments(const double2* x, int64_t xstride, const double* m1, int q, int d, int p, int L,
                             int k, int64_t leaf_off, int64_t nleaf, double2* xh, int deriv_u, int deriv_v,
                             int64_t m1_stride_kind, int ncol) {
    const int nq = (q + 1) * (q + 1);
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= nleaf * nq * ncol) return;
    const int r = int(gid % ncol);
    const int64_t t = gid / ncol;
    const int64_t c = t / nq;
    const int a = int(t % nq), au = a % (q + 1), av = a / (q + 1);
    const int n = 1 << L, s = 1 << d, w = s + p;
    const int patch = int(c / (int64_t(n) * n));
    const int rem = int(c % (int64_t(n) * n));
    const int cy = rem / n, cx = rem % n;
    const double* mu = m1 + deriv_u * m1_stride_kind + (int64_t(cx) * (q + 1) + au) * w;
    const double* mv = m1 + deriv_v * m1_stride_kind + (int64_t(cy) * (q + 1) + av) * w;
    const double2* X = x + r * xstride + int64_t(patch) * k * k + int64_t(cy) * s * k + int64_t(cx) * s;
    double2 acc = make_double2(0, 0);
    for (int iv = 0; iv < w; ++iv) {
        double2 row = make_double2(0, 0);
        for (int iu = 0; iu < w; ++iu) {
            const double2 xv = X[int64_t(iv) * k + iu];
            row.x = fma(mu[iu], xv.x, row.x);
            row.y = fma(mu[iu], xv.y, row.y);
        }
        acc.x = fma(mv[iv], row.x, acc.x);
        acc.y = fma(mv[iv], row.y, acc.y);
    }
    xh[((leaf_off + c) * nq + a) * ncol + r] = acc;
}

// ---- workgroup-per-cluster tree kernels (LDS staged, sum-factorised) ----
constexpr int TREE_THREADS = 128;
constexpr int TQ1 = QMAX + 1;
constexpr int TNQ = TQ1 * TQ1;

// upward, one workgroup per (parent at level l, block of cb columns):
//   x^_P[av][au] = sum_c sum_gv Tv_c[gv][av] sum_gu Tu_c[gu][au] x^_c[gv][gu]
// (dynamic LDS: the children's moments and the half-transferred values,
// 4 (q+1)^2 cb each, columns fastest; each column's operations and their order
// do not depend on cb)
__global__ __launch_bounds__(256) void m2m_wg(const double* __restrict__ T1, int q, int l, int64_t off_l,
                                              int64_t off_l1, double2* xh, int ncol, int cb) {
    extern __shared__ double2 dyn[];
    __shared__ double T[2 * TQ1 * TQ1];
    const int q1 = q + 1, nq = q1 * q1, tid = threadIdx.x, nt = blockDim.x;
    double2* X = dyn;
    double2* tmp = dyn + 4 * nq * cb;
    const int64_t c = blockIdx.x;
    const int c0 = blockIdx.y * cb;
    const int n = 1 << l;
    const int patch = int(c / (int64_t(n) * n));
    const int rem = int(c % (int64_t(n) * n));
    const int cy = rem / n, cx = rem % n;
    for (int i = tid; i < 2 * q1 * q1; i += nt) T[i] = T1[i];
    for (int i = tid; i < 4 * nq * cb; i += nt) {
        const int k = i % cb, t = i / cb, ch = t / nq, a = t % nq, bu = ch & 1, bv = ch >> 1;
        const int64_t child = off_l1 + (int64_t(patch) << (2 * (l + 1))) + (int64_t(2 * cy + bv) << (l + 1)) +
                              2 * cx + bu;
        X[i] = c0 + k < ncol ? xh[(child * nq + a) * ncol + c0 + k] : make_double2(0, 0);
    }
    __syncthreads();
    for (int i = tid; i < 4 * nq * cb; i += nt) {
        const int k = i % cb, t = i / cb, ch = t / nq, r = t % nq, gv = r / q1, au = r % q1, bu = ch & 1;
        const double* Tu = T + bu * q1 * q1;
        double2 acc = make_double2(0, 0);
        for (int gu = 0; gu < q1; ++gu) {
            const double tt = Tu[gu * q1 + au];
            const double2 xv = X[(ch * nq + gv * q1 + gu) * cb + k];
            acc.x = fma(tt, xv.x, acc.x);
            acc.y = fma(tt, xv.y, acc.y);
        }
        tmp[i] = acc;
    }
    __syncthreads();
    for (int i = tid; i < nq * cb; i += nt) {
        const int k = i % cb, a = i / cb, av = a / q1, au = a % q1;
        if (c0 + k >= ncol) continue;
        double2 acc = make_double2(0, 0);
        for (int ch = 0; ch < 4; ++ch) {
            const double* Tv = T + (ch >> 1) * q1 * q1;
            for (int gv = 0; gv < q1; ++gv) {
                const double tt = Tv[gv * q1 + av];
                const double2 v = tmp[(ch * nq + gv * q1 + au) * cb + k];
                acc.x = fma(tt, v.x, acc.x);
                acc.y = fma(tt, v.y, acc.y);
            }
        }
        xh[((off_l + c) * nq + a) * ncol + c0 + k] = acc;
    }
}

// the upward pass above the leaves: m2m_wg level by level, up to 8 columns per
// workgroup within 48 KB of dynamic LDS
// levels L-1 down to lmin (the coarser ones are not needed)
static void launch_m2m_levels(const double* T1, int q, int L, int npatch, const std::vector<int64_t>& clu_off,
                              double2* xh, int ncol, hipStream_t s, int lmin = 0) {
    const int nq = (q + 1) * (q + 1);
    int cb = std::min(ncol, 8);
    while (cb > 2 && size_t(8) * nq * cb * sizeof(double2) > 48 * 1024) cb /= 2;
    const size_t lds = size_t(8) * nq * cb * sizeof(double2);
    const unsigned cblk = unsigned((ncol + cb - 1) / cb);
    for (int l = L - 1; l >= std::max(lmin, 0); --l)
        hipLaunchKernelGGL(m2m_wg, dim3(unsigned(clusters_on_level(npatch, l)), cblk), dim3(cb >= 4 ? 256 : TREE_THREADS),
                           lds, s, T1, q, l, clu_off[l], clu_off[l + 1], xh, ncol, cb);
}

// The far part of the product at S^2 index i and column r, gathered from the
// leaf buffers of the downward pass: the sum over the leaves whose B-spline
// windows hold i (and over the moment kinds), in a fixed order.  The near
// kernels add it to each row after the row's near sum.
struct FarLeaves {
    const double2* leafbuf;   // null: no far part
    int d, p, L, k, npatch, kinds, ncol;
};
__device__ __forceinline__ double2 far_value(const FarLeaves& F, int64_t i, int r) {
    const int64_t kk = int64_t(F.k) * F.k;
    const int patch = int(i / kk);
    const int rem = int(i % kk);
    const int iv = rem / F.k, iu = rem % F.k;
    const int s = 1 << F.d, w = s + F.p, n = 1 << F.L;
    const int64_t nleaf = int64_t(F.npatch) * n * n;
    double2 acc = make_double2(0, 0);
    const int cy0 = max(0, (iv - w + s) / s), cy1 = min(n - 1, iv / s);
    const int cx0 = max(0, (iu - w + s) / s), cx1 = min(n - 1, iu / s);
    for (int cy = cy0; cy <= cy1; ++cy) {
        const int lv = iv - cy * s;
        if (lv < 0 || lv >= w) continue;
        for (int cx = cx0; cx <= cx1; ++cx) {
            const int lu = iu - cx * s;
            if (lu < 0 || lu >= w) continue;
            const int64_t leaf = (int64_t(patch) << (2 * F.L)) + int64_t(cy) * n + cx;
            for (int kd = 0; kd < F.kinds; ++kd)
                acc = cadd(acc, F.leafbuf[((kd * nleaf + leaf) * F.ncol + r) * w * w + lv * w + lu]);
        }
    }
    return acc;
}

// storage types of the coupling tiles: fp64, fp32 or bf16 complex; products and
// accumulation run in fp64 on the VALU path
struct bf16x2 {
    unsigned short re, im;
};
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 to_d2(bf16x2 v) {
    return make_double2(__uint_as_float(unsigned(v.re) << 16), __uint_as_float(unsigned(v.im) << 16));
}
__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// downward pass and back projection in one launch, one workgroup per leaf and
// block of columns: the leaf's local expansion collects every ancestor's
// (each read as the sum of its coupling partials when those are given),
//   y^_leaf += (Tv ⊗ Tu)_(delta, pos) y^_A   for the ancestors A, nearest first,
// with the composite transfers Tc[delta][pos][g][a] = L_a((pos + t_g) / 2^delta)
// (the ancestor's Lagrange basis at the leaf's nodes, delta levels down at
// offset pos; interpolating a degree-q expansion again at finer nodes is
// exact, so this equals the level-by-level pass), then is back projected
// onto the leaf's (s+p)^2 window:
//   out[lv][lu] = sum_av m_v[av][lv] sum_au m_u[au][lu] y^[av][au]
// (cb columns per workgroup share the transfers' loads; each column's
// operations and their order do not depend on cb.  Dynamic LDS: y^, the
// ancestor's y^ and the half-transferred values, cb x (q+1)^2 each, then the
// half-projected values cb x (q+1) x w; node-major, columns fastest.)
template <class PT>
__global__ __launch_bounds__(256) void down_project_leaf(const double2* __restrict__ yh,
                                                         const PT* __restrict__ part,
                                                         const int* __restrict__ chunk_ptr,
                                                         const double* __restrict__ Tc,
                                                         const int64_t* __restrict__ clu_off,
                                                         const double* __restrict__ m1, int q, int w, int L,
                                                         int lmin, int deriv_u, int deriv_v,
                                                         int64_t m1_stride_kind, int ncol, int cb,
                                                         double2* __restrict__ leafbuf) {
    extern __shared__ double2 dyn[];
    __shared__ double Mu[TQ1 * TQ1], Mv[TQ1 * TQ1];
    const int q1 = q + 1, nq = q1 * q1, tid = threadIdx.x, nt = blockDim.x;
    const int64_t c = blockIdx.x;
    const int r0 = blockIdx.y * cb, nr = min(cb, ncol - r0);
    double2* Y = dyn;
    double2* YA = Y + cb * nq;
    double2* tmp = YA + cb * nq;
    double2* tb = tmp + cb * nq;
    const int n = 1 << L;
    const int patch = int(c / (int64_t(n) * n));
    const int rem = int(c % (int64_t(n) * n));
    const int cy = rem / n, cx = rem % n;
    // y^ of cluster X at node e, column r: the sum of its coupling chunks' partials
    // (in chunk order, as m2l_reduce forms it) or, without partials, y^ itself
    auto yget = [&](int64_t X, int e, int r) {
        if (!part) return yh[(X * nq + e) * ncol + r];
        double2 acc = make_double2(0, 0);
        for (int ch = chunk_ptr[X]; ch < chunk_ptr[X + 1]; ++ch)
            acc = cadd(acc, to_d2(part[(int64_t(ch) * nq + e) * ncol + r]));
        return acc;
    };
    for (int i = tid; i < nq * nr; i += nt) Y[i] = yget(clu_off[L] + c, i / nr, r0 + i % nr);
    // ancestors coarser than lmin hold no coupling results
    for (int l = L - 1; l >= lmin; --l) {
        const int dl = L - l, msk = (1 << dl) - 1;
        const int64_t A = clu_off[l] + (int64_t(patch) << (2 * l)) + (int64_t(cy >> dl) << l) + (cx >> dl);
        const double* Tu = Tc + int64_t((1 << dl) - 2 + (cx & msk)) * q1 * q1;
        const double* Tv = Tc + int64_t((1 << dl) - 2 + (cy & msk)) * q1 * q1;
        __syncthreads();   // previous ancestor's YA / tmp consumed
        for (int i = tid; i < nq * nr; i += nt) YA[i] = yget(A, i / nr, r0 + i % nr);
        for (int i = tid; i < nq; i += nt) {
            Mu[i] = Tu[i];
            Mv[i] = Tv[i];
        }
        __syncthreads();
        // tmp[av][gu] = sum_au Tu[gu][au] y^_A[av][au]
        for (int i = tid; i < nq * nr; i += nt) {
            const int k = i % nr, e = i / nr, av = e / q1, gu = e % q1;
            double2 acc = make_double2(0, 0);
            for (int au = 0; au < q1; ++au) {
                const double t = Mu[gu * q1 + au];
                const double2 v = YA[(av * q1 + au) * nr + k];
                acc.x = fma(t, v.x, acc.x);
                acc.y = fma(t, v.y, acc.y);
            }
            tmp[i] = acc;
        }
        __syncthreads();
        // y^[gv][gu] += sum_av Tv[gv][av] tmp[av][gu]
        for (int i = tid; i < nq * nr; i += nt) {
            const int k = i % nr, e = i / nr, gv = e / q1, gu = e % q1;
            double2 acc = make_double2(0, 0);
            for (int av = 0; av < q1; ++av) {
                const double t = Mv[gv * q1 + av];
                const double2 v = tmp[(av * q1 + gu) * nr + k];
                acc.x = fma(t, v.x, acc.x);
                acc.y = fma(t, v.y, acc.y);
            }
            Y[i] = cadd(Y[i], acc);
        }
    }
    __syncthreads();
    const double* mu = m1 + deriv_u * m1_stride_kind + int64_t(cx) * q1 * w;
    const double* mv = m1 + deriv_v * m1_stride_kind + int64_t(cy) * q1 * w;
    for (int i = tid; i < q1 * w * nr; i += nt) {
        const int k = i % nr, e = i / nr, av = e / w, lu = e % w;
        double2 acc = make_double2(0, 0);
        for (int au = 0; au < q1; ++au) {
            const double t = mu[au * w + lu];
            const double2 v = Y[(av * q1 + au) * nr + k];
            acc.x = fma(t, v.x, acc.x);
            acc.y = fma(t, v.y, acc.y);
        }
        tb[i] = acc;
    }
    __syncthreads();
    for (int i = tid; i < w * w * nr; i += nt) {
        const int k = i / (w * w), e = i % (w * w), lv = e / w, lu = e % w;
        double2 acc = make_double2(0, 0);
        for (int av = 0; av < q1; ++av) {
            const double t = mv[av * w + lv];
            const double2 v = tb[(av * w + lu) * nr + k];
            acc.x = fma(t, v.x, acc.x);
            acc.y = fma(t, v.y, acc.y);
        }
        leafbuf[(c * ncol + r0 + k) * w * w + e] = acc;
    }
}

// columns per workgroup of down_project_leaf: up to 8, within 48 KB of dynamic LDS
static inline int down_cols(int ncol, int q1, int w, size_t& lds) {
    int cb = std::min(ncol, 8);
    auto bytes = [&](int k) { return size_t(k) * (3 * q1 * q1 + q1 * w) * sizeof(double2); };
    while (cb > 1 && bytes(cb) > 48 * 1024) cb /= 2;
    lds = bytes(cb);
    return cb;
}


// ---------------------------------------------------------------------------
// Reduced-precision coupling on the matrix cores
//
// The complex products y[a][c] += sum_b K[a][b] x[b][c] of one coupling tile
// run as one real GEMM with fp32 accumulation: the tile, row-major with (re,
// im) adjacent, is the A operand A'[a][2b + r]; the B operand comes from the
// compact source vector, (Re x, -Im x) along k for Re y and (Im x, Re x) for
// Im y.  Both operands are stored in 16-byte chunks of EPL consecutive
// elements (element = bf16 or fp32 complex) so that the 16 lanes of a lane
// group, which hold 16 consecutive rows (A) or columns (B) of one chunk, read
// 256 contiguous bytes:
//   tiles    [pair][tile][chunk kc < nkc][row a < nq][EPL], nkc = ceil(nq/EPL),
//            zeros beyond nq (tile 0: soft kernel or hard G, tile 1: hard H)
//   vectors  [cluster][vec][chunk < kbp/EPL][col < ncolp][EPL], kbp = nq
//            rounded up to the k block, ncolp = ncol rounded up to 16, zeros
//            beyond nq and ncol
// The last k block of a tile may cover up to three chunks past nq: the A
// reads of those lanes are clamped to the tile's last chunk (already cached)
// and the B operand is zero there.
// ---------------------------------------------------------------------------
template <class LT> __device__ __forceinline__ LT round_to(double2 v);
template <> __device__ __forceinline__ float2 round_to<float2>(double2 v) { return make_float2(float(v.x), float(v.y)); }
template <> __device__ __forceinline__ double2 round_to<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ bf16x2 round_to<bf16x2>(double2 v) {
    bf16x2 b;
    b.re = f32_to_bf16_rne(float(v.x));   // RNE of the fp32 value
    b.im = f32_to_bf16_rne(float(v.y));
    return b;
}

// rounded tiles in matrix-core order, each entry evaluated in fp64 by the same
// functions as the fp64 tiles and rounded once (no fp64 tiles needed)
template <class LT, bool HARD>
__global__ void coupling_lo(const double* __restrict__ nodes, const int* __restrict__ pair_tgt,
                            const int* __restrict__ pair_src, int64_t nfar, int nq, int nkc, double kappa, SoftMix mix,
                            LT* __restrict__ out) {
    constexpr int EPL = 16 / sizeof(LT), NT = HARD ? 2 : 1;
    const int64_t total = nfar * NT * nkc * nq * EPL;
    // grid-stride: the tiles of a large operator exceed the 2^32 threads of a grid
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
    const int e = int(i % EPL);
    int64_t r = i / EPL;
    const int a = int(r % nq);
    r /= nq;
    const int kc = int(r % nkc);
    r /= nkc;
    const int t = int(r % NT);
    const int64_t pr = r / NT;
    const int b = kc * EPL + e;
    double2 v = make_double2(0, 0);
    if (b < nq) {
        const double* X = nodes + (int64_t(pair_tgt[pr]) * nq + a) * 16;
        const double* Y = nodes + (int64_t(pair_src[pr]) * nq + b) * 16;
        if (HARD) {
            double2 G, H;
            kernel_gh(X, Y, kappa, G, H);
            v = t == 0 ? G : H;
        } else {
            v = kernel_soft(X, X + 3, X[6], Y, Y[6], kappa, mix);
        }
    }
    out[i] = round_to<LT>(v);
    }
}

// rounded source vectors of the coupling, per matvec.  Soft: the moments x.
// Hard (NV = 7): n~_c xp (c = 0..2), (y.n~) xp, F_v,c xu - F_u,c xv (c = 0..2)
// at the cluster's nodes, from the three moment kinds xp, xu, xv.
template <int NV, class LT>
__global__ void round_vectors(const double2* __restrict__ xh, int64_t ks, const double* __restrict__ nodes,
                              int64_t nclusters, int nq, int kbp, int ncol, int ncolp, LT* __restrict__ out) {
    constexpr int EPL = 16 / sizeof(LT);
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nclusters * NV * ncolp * kbp) return;
    const int e = int(i % EPL);
    int64_t r = i / EPL;
    const int c = int(r % ncolp);
    r /= ncolp;
    const int nch = kbp / EPL;
    const int kc = int(r % nch);
    r /= nch;
    const int v = int(r % NV);
    const int64_t cl = r / NV;
    const int b = kc * EPL + e;
    double2 val = make_double2(0, 0);
    if (b < nq && c < ncol) {
        const int64_t o = (cl * nq + b) * ncol + c;
        if (NV == 1) {
            val = xh[o];
        } else {
            const double* Y = nodes + (cl * nq + b) * 16;
            if (v < 3) {
                val = cscale(xh[o], Y[3 + v]);
            } else if (v == 3) {
                val = cscale(xh[o], Y[0] * Y[3] + Y[1] * Y[4] + Y[2] * Y[5]);
            } else {
                const int cc = v - 4;
                const double2 xu = xh[ks + o], xv = xh[2 * ks + o];
                val = make_double2(Y[11 + cc] * xu.x - Y[8 + cc] * xv.x, Y[11 + cc] * xu.y - Y[8 + cc] * xv.y);
            }
        }
    }
    out[i] = round_to<LT>(val);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));

// One k block of one 16x16 output tile.  Each lane holds 16 bytes of A (row
// lane%16) and of B (column lane%16); lane group g = lane/16 holds the k
// entries g*KB/4 .. of the block.  Any assignment of k to register slots is
// valid as long as A and B use the same one, which they do by construction.
struct MfmaBf16 {
    using LT = bf16x2;
    using ACC = f32x4;
    using PT = float2;
    // output row of register r in lane group g (column = lane % 16)
    static __device__ __forceinline__ int orow(int g, int r) { return 4 * g + r; }
    static constexpr int EPL = 4;    // complex elements per lane load
    static constexpr int KB = 16;    // complex elements per k block (k = 32)
    static __device__ __forceinline__ f32x4 step(uint4 a, uint4 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8v, a), __builtin_bit_cast(bf16x8v, b),
                                                       c, 0, 0, 0);
    }
    static __device__ __forceinline__ uint4 re_part(uint4 x) {   // (re, im) -> (re, -im)
        return make_uint4(x.x ^ 0x80000000u, x.y ^ 0x80000000u, x.z ^ 0x80000000u, x.w ^ 0x80000000u);
    }
    static __device__ __forceinline__ uint4 im_part(uint4 x) {   // (re, im) -> (im, re)
        return make_uint4((x.x >> 16) | (x.x << 16), (x.y >> 16) | (x.y << 16), (x.z >> 16) | (x.z << 16),
                          (x.w >> 16) | (x.w << 16));
    }
};
struct MfmaF32 {
    using LT = float2;
    using ACC = f32x4;
    using PT = float2;
    static __device__ __forceinline__ int orow(int g, int r) { return 4 * g + r; }
    static constexpr int EPL = 2;
    static constexpr int KB = 8;     // four 16x16x4 steps
    static __device__ __forceinline__ f32x4 step(uint4 a, uint4 b, f32x4 c) {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
        return c;
    }
    static __device__ __forceinline__ uint4 re_part(uint4 x) {   // (re0, im0, re1, im1) -> (re0, -im0, re1, -im1)
        return make_uint4(x.x, x.y ^ 0x80000000u, x.z, x.w ^ 0x80000000u);
    }
    static __device__ __forceinline__ uint4 im_part(uint4 x) {   // -> (im0, re0, im1, re1)
        return make_uint4(x.y, x.x, x.w, x.z);
    }
};

// fp64: one complex (16 bytes) per lane and k block of 4 complex; each lane
// group's complex supplies the re part to the first 16x16x4 step and the im
// part to the second
typedef double f64x4 __attribute__((ext_vector_type(4)));
struct MfmaF64 {
    using LT = double2;
    using ACC = f64x4;
    using PT = double2;
    // the fp64 16x16x4 instruction interleaves its output rows across registers
    static __device__ __forceinline__ int orow(int g, int r) { return g + 4 * r; }
    static constexpr int EPL = 1;
    static constexpr int KB = 4;
    static __device__ __forceinline__ double lo(uint4 v) {
        return __longlong_as_double((long long)(((unsigned long long)v.y << 32) | v.x));
    }
    static __device__ __forceinline__ double hi(uint4 v) {
        return __longlong_as_double((long long)(((unsigned long long)v.w << 32) | v.z));
    }
    static __device__ __forceinline__ f64x4 step(uint4 a, uint4 b, f64x4 c) {
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(lo(a), lo(b), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(hi(a), hi(b), c, 0, 0, 0);
        return c;
    }
    static __device__ __forceinline__ uint4 re_part(uint4 x) {   // (re, im) -> (re, -im)
        return make_uint4(x.x, x.y, x.z, x.w ^ 0x80000000u);
    }
    static __device__ __forceinline__ uint4 im_part(uint4 x) {   // -> (im, re)
        return make_uint4(x.z, x.w, x.x, x.y);
    }
};
template <class PT> __device__ __forceinline__ PT make_pt(double re, double im);
template <> __device__ __forceinline__ float2 make_pt<float2>(double re, double im) {
    return make_float2(float(re), float(im));
}
template <> __device__ __forceinline__ double2 make_pt<double2>(double re, double im) {
    return make_double2(re, im);
}

// chunk handled by workgroup w: consecutive chunks on the same XCD (workgroups
// are dealt to the 8 XCDs round robin), so neighbouring targets share L2
__device__ __forceinline__ int64_t xcd_chunk(int64_t w, int64_t n) {
    const int64_t per = n / 8, rem = n % 8, x = w % 8, i = w / 8;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// matrix-core layout sizes of the operator's own precision (fp64 operators use
// the fp64 tiles [pair][tile][b][a], which are the chunk layout with EPL = 1)
static inline int lo_kb(igb_op op) {
    return op->prm.precision == IGB_MIX_FP32 ? MfmaF32::KB : op->prm.precision == IGB_MIX_BF16 ? MfmaBf16::KB : MfmaF64::KB;
}
static inline int lo_epl(igb_op op) {
    return op->prm.precision == IGB_MIX_FP32 ? MfmaF32::EPL
                                              : op->prm.precision == IGB_MIX_BF16 ? MfmaBf16::EPL : MfmaF64::EPL;
}
static inline int lo_nkc(igb_op op) { return (op->nq + lo_epl(op) - 1) / lo_epl(op); }
static inline int lo_kbp(igb_op op) { return (op->nq + lo_kb(op) - 1) / lo_kb(op) * lo_kb(op); }
// k extent of the fp64 matrix-core source vectors (the on-the-fly coupling's)
static inline int kbp_f64(int nq) { return (nq + MfmaF64::KB - 1) / MfmaF64::KB * MfmaF64::KB; }
static inline size_t lo_esz(igb_op op) {
    return op->prm.precision == IGB_MIX_FP32 ? sizeof(float2)
                                              : op->prm.precision == IGB_MIX_BF16 ? sizeof(bf16x2) : sizeof(double2);
}
// the matrix-core coupling serves the operator's own precision; an fp64
// operator with tiles uses it for every product
static inline bool mf_fp64(igb_op op) { return op->prm.precision == IGB_FP64 && !op->prm.far_on_the_fly; }
// zeroed guard bytes after the last tile (A reads are clamped to the tile)
static inline size_t lo_slack(igb_op op) { return size_t(3) * op->nq * 16 + 256; }

// Coupling of one chunk (consecutive far pairs of one target) for 16 columns
// on the matrix cores: wave w owns the RPW output row tiles RPW w .. RPW w +
// RPW - 1 (16 rows each), so the source fragments a wave loads per step serve
// RPW row tiles.  Soft: one tile, one vector.  Hard: H acts on vectors
// {3, 0, 1, 2}, G on {0, 1, 2, 4, 5, 6}, giving the 10 partial vectors of the
// vector-path kernel in the same order.  Each output row's operations and
// their order do not depend on RPW.
constexpr int M2L_RPW = 3;   // row tiles per wave of m2l_mfma (fp32 / bf16)
template <class OPS, bool HARD, int RPW = 1>
__global__ __launch_bounds__(512 / RPW) void m2l_mfma(const typename OPS::LT* __restrict__ coup, int nkc,
                                                const typename OPS::LT* __restrict__ xlo, int kbp, int ncolp,
                                                const int* __restrict__ far_src_g,
                                                const int64_t* __restrict__ chunk_pair,
                                                const int* __restrict__ chunk_len, int64_t nchunk, int nq, int ncol,
                                                typename OPS::PT* __restrict__ part) {
    constexpr int NT = HARD ? 2 : 1, NVS = HARD ? 7 : 1, NVO = HARD ? 10 : 1;
    constexpr int KB = OPS::KB, EPL = OPS::EPL;
    const int64_t ch = xcd_chunk(blockIdx.x, nchunk);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    // A rows of this lane; rows past nq re-read the last row (their outputs are
    // not stored, and an output row depends only on its own A row)
    int a[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) a[k] = min((wave * RPW + k) * 16 + li, nq - 1);
    const int c0 = blockIdx.y * 16;
    const int64_t p0 = chunk_pair[ch];
    const int len = chunk_len[ch];
    const int nkb = (nq + KB - 1) / KB;
    const int64_t tile_el = int64_t(nkc) * nq * EPL;
    using ACC = typename OPS::ACC;
    ACC acc[RPW][NVO][2];
#pragma unroll
    for (int k = 0; k < RPW; ++k)
#pragma unroll
        for (int v = 0; v < NVO; ++v) acc[k][v][0] = acc[k][v][1] = ACC{0, 0, 0, 0};
    // steps j = (pair i, k block kb) in order; KU steps issue their loads
    // before any of their products, so each wave keeps KU blocks in flight.
    // (Sound-hard, one wave per SIMD: two steps in flight instead of one took
    // the bf16 coupling of the level-6 hard star from 1.11 to 0.68 ms; the fp64
    // form, two waves per SIMD, would spill.)
    constexpr int KU = HARD ? (std::is_same<OPS, MfmaF64>::value ? 1 : 2) : 4;
    const int nstep = len * nkb;
    // the chunk's source clusters, lane i holding pair i (len <= 64), read back
    // with readlane: no dependent scalar load inside the loop
    const int srcv = lane < len ? far_src_g[p0 + lane] : 0;
    const int64_t vstride = int64_t(ncolp) * kbp;
    // addresses: a uniform part per step (scalar unit) plus a per-lane 32-bit
    // offset fixed for the whole kernel
    using LT = typename OPS::LT;
    unsigned offA[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) offA[k] = unsigned(a[k] * EPL);
    const unsigned offB = unsigned((g * ncolp + c0 + li) * EPL);
    // next step to load: pair ni, k block nkbi.  Past the last step the loads
    // repeat the last step's (in bounds, unused): every load is issued
    // unconditionally, so the compiler can wait for exactly the buffer a group
    // of products needs while the other buffer's loads stay in flight.
    int ni = 0, nkbi = 0;
    auto load = [&](uint4 (&A)[KU][RPW][NT], uint4 (&X)[KU][NVS]) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int i = ni, kb = nkbi;
            const bool last = ni == len - 1 && nkbi == nkb - 1;
            nkbi = last ? nkbi : (nkbi + 1 == nkb ? 0 : nkbi + 1);
            ni = last ? ni : (nkbi == 0 ? ni + 1 : ni);
            const int src = __builtin_amdgcn_readlane(srcv, i);
            // chunk of this lane group, clamped to the tile: past nq the B operand
            // is zero, and a re-read chunk of the same tile is already cached
            const int kcg = min(kb * 4 + g, nkc - 1);
            const LT* Au = coup + (p0 + i) * (NT * tile_el) + int64_t(kcg) * nq * EPL;
            const LT* Bu = xlo + int64_t(src) * (NVS * vstride) + kb * (4 * ncolp * EPL);
#pragma unroll
            for (int k = 0; k < RPW; ++k)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    A[u][k][t] = *reinterpret_cast<const uint4*>(Au + t * tile_el + offA[k]);
#pragma unroll
            for (int v = 0; v < NVS; ++v) X[u][v] = *reinterpret_cast<const uint4*>(Bu + v * vstride + offB);
        }
    };
    auto compute = [&](int j0, const uint4 (&A)[KU][RPW][NT], const uint4 (&X)[KU][NVS]) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            if (j0 + u >= nstep) break;
#pragma unroll
            for (int k = 0; k < RPW; ++k) {
                if constexpr (!HARD) {
                    acc[k][0][0] = OPS::step(A[u][k][0], OPS::re_part(X[u][0]), acc[k][0][0]);
                    acc[k][0][1] = OPS::step(A[u][k][0], OPS::im_part(X[u][0]), acc[k][0][1]);
                } else {
                    constexpr int hv[4] = {3, 0, 1, 2};
                    constexpr int gv[6] = {0, 1, 2, 4, 5, 6};
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        acc[k][jj][0] = OPS::step(A[u][k][1], OPS::re_part(X[u][hv[jj]]), acc[k][jj][0]);
                        acc[k][jj][1] = OPS::step(A[u][k][1], OPS::im_part(X[u][hv[jj]]), acc[k][jj][1]);
                    }
#pragma unroll
                    for (int jj = 0; jj < 6; ++jj) {
                        acc[k][4 + jj][0] = OPS::step(A[u][k][0], OPS::re_part(X[u][gv[jj]]), acc[k][4 + jj][0]);
                        acc[k][4 + jj][1] = OPS::step(A[u][k][0], OPS::im_part(X[u][gv[jj]]), acc[k][4 + jj][1]);
                    }
                }
            }
        }
    };
    // two register buffers: the next group's loads are in flight while the
    // current group's products run
    uint4 A0[KU][RPW][NT], X0[KU][NVS], A1[KU][RPW][NT], X1[KU][NVS];
    load(A0, X0);
    for (int j0 = 0; j0 < nstep; j0 += 2 * KU) {
        load(A1, X1);
        compute(j0, A0, X0);
        load(A0, X0);
        compute(j0 + KU, A1, X1);
    }
    // lane holds column li and rows OPS::orow(g, 0..3) of each 16x16 tile
    const int c = c0 + li;
    if (c >= ncol) return;
#pragma unroll
    for (int k = 0; k < RPW; ++k)
#pragma unroll
        for (int v = 0; v < NVO; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ar = (wave * RPW + k) * 16 + OPS::orow(g, r);
                if (ar < nq)
                    part[((ch * NVO + v) * nq + ar) * ncol + c] =
                        make_pt<typename OPS::PT>(acc[k][v][0][r], acc[k][v][1][r]);
            }
}

// fp64 sound-soft coupling for blocks of >= 16 columns on the fp64 matrix
// cores, with A reuse: wave w owns output rows 16w..16w+15 of the chunk's
// target and NC tiles of 16 columns, so every A fragment (16 rows x 4 source
// nodes of one tile) read from HBM serves NC column tiles (the coupling of 64
// columns reads each tile once: arithmetic intensity 32 flop/B, past the fp64
// ridge).  The waves of a workgroup read the same source fragments, which the
// cache serves once.  Each column sums the chunk's pairs and k blocks in
// order in its own accumulator, so its result does not depend on NC or on the
// other columns.  KU steps are loaded per group, two groups in flight.
template <int NC, int KU>
__global__ __launch_bounds__(512) void m2l_mfma64_soft(const double2* __restrict__ coup, int nkc,
                                                       const double2* __restrict__ xlo, int kbp, int ncolp,
                                                       const int* __restrict__ far_src_g,
                                                       const int64_t* __restrict__ chunk_pair,
                                                       const int* __restrict__ chunk_len, int64_t nchunk, int nq,
                                                       int ncol, double2* __restrict__ part) {
    using OPS = MfmaF64;
    constexpr int KB = OPS::KB;
    const int64_t ch = xcd_chunk(blockIdx.x, nchunk);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    // A row of this lane; rows past nq re-read the last row (outputs not stored)
    const int a = min(wave * 16 + li, nq - 1);
    const int c0 = blockIdx.y * 16 * NC;
    const int64_t p0 = chunk_pair[ch];
    const int len = chunk_len[ch];
    const int nkb = (nq + KB - 1) / KB;
    const int64_t tile_el = int64_t(nkc) * nq;
    const int nstep = len * nkb;
    const int srcv = lane < len ? far_src_g[p0 + lane] : 0;
    const int64_t vstride = int64_t(ncolp) * kbp;
    const unsigned offB = unsigned(g * ncolp + c0 + li);
    OPS::ACC acc[NC][2];
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j][0] = acc[j][1] = OPS::ACC{0, 0, 0, 0};
    // next step to load; past the last step the loads repeat it (in bounds,
    // unused), so every load is issued unconditionally
    int ni = 0, nkbi = 0;
    auto load = [&](uint4 (&A)[KU], uint4 (&X)[KU][NC]) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int i = ni, kb = nkbi;
            const bool last = ni == len - 1 && nkbi == nkb - 1;
            nkbi = last ? nkbi : (nkbi + 1 == nkb ? 0 : nkbi + 1);
            ni = last ? ni : (nkbi == 0 ? ni + 1 : ni);
            const int src = __builtin_amdgcn_readlane(srcv, i);
            const int kcg = min(kb * KB + g, nkc - 1);   // clamped to the tile (B is zero past nq)
            A[u] = *reinterpret_cast<const uint4*>(coup + (p0 + i) * tile_el + int64_t(kcg) * nq + a);
            const double2* Bu = xlo + int64_t(src) * vstride + kb * (KB * ncolp) + offB;
#pragma unroll
            for (int j = 0; j < NC; ++j) X[u][j] = *reinterpret_cast<const uint4*>(Bu + 16 * j);
        }
    };
    auto compute = [&](int j0, const uint4 (&A)[KU], const uint4 (&X)[KU][NC]) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            if (j0 + u >= nstep) break;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                acc[j][0] = OPS::step(A[u], OPS::re_part(X[u][j]), acc[j][0]);
                acc[j][1] = OPS::step(A[u], OPS::im_part(X[u][j]), acc[j][1]);
            }
        }
    };
    uint4 A0[KU], X0[KU][NC], A1[KU], X1[KU][NC];
    load(A0, X0);
    for (int j0 = 0; j0 < nstep; j0 += 2 * KU) {
        load(A1, X1);
        compute(j0, A0, X0);
        load(A0, X0);
        compute(j0 + KU, A1, X1);
    }
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        const int c = c0 + 16 * j + li;
        if (c >= ncol) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ar = wave * 16 + OPS::orow(g, r);
            if (ar < nq) part[(ch * nq + ar) * ncol + c] = make_double2(acc[j][0][r], acc[j][1][r]);
        }
    }
}

// Sound-soft coupling on the matrix cores with B reuse: the 4 waves of a
// workgroup take every 4th pair of the chunk, and each wave computes all MT
// row tiles of its pairs, so one B fragment per k block serves MT products.
// The waves' sums meet in LDS and are added in wave order (fixed).
template <class OPS, int MT>
__global__ __launch_bounds__(256) void m2l_mfma_soft(const typename OPS::LT* __restrict__ coup, int nkc,
                                                     const typename OPS::LT* __restrict__ xlo, int kbp, int ncolp,
                                                     const int* __restrict__ far_src_g,
                                                     const int64_t* __restrict__ chunk_pair,
                                                     const int* __restrict__ chunk_len, int64_t nchunk, int nq,
                                                     int ncol, typename OPS::PT* __restrict__ part) {
    using LT = typename OPS::LT;
    constexpr int KB = OPS::KB, EPL = OPS::EPL, NW = 4;
    using ACC = typename OPS::ACC;
    __shared__ ACC red[NW - 1][MT][2][64];
    const int64_t ch = xcd_chunk(blockIdx.x, nchunk);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    const int c0 = blockIdx.y * 16;
    const int64_t p0 = chunk_pair[ch];
    const int len = chunk_len[ch];
    const int nkb = (nq + KB - 1) / KB;
    const int64_t tile_el = int64_t(nkc) * nq * EPL;
    const int64_t vstride = int64_t(ncolp) * kbp;
    const int srcv = lane < len ? far_src_g[p0 + lane] : 0;
    // lane offsets: rows past nq re-read row nq-1 (outputs not stored)
    unsigned offA[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) offA[mt] = unsigned(min(mt * 16 + li, nq - 1) * EPL);
    const unsigned offB = unsigned((g * ncolp + c0 + li) * EPL);
    ACC acc[MT][2];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt][0] = acc[mt][1] = ACC{0, 0, 0, 0};
    // this wave's steps: pairs wave, wave+4, ..., k blocks 0..nkb-1; loads past
    // the last step repeat it (in bounds, unused) so they are unconditional
    const int npair = len > wave ? (len - wave + NW - 1) / NW : 0;
    const int nstep = npair * nkb;
    int ni = 0, nkbi = 0;
    auto load = [&](uint4 (&A)[MT], uint4& X) {
        const int i = wave + NW * min(ni, max(npair - 1, 0)), kb = nkbi;
        const bool last = ni >= npair - 1 && nkbi == nkb - 1;
        nkbi = last ? nkbi : (nkbi + 1 == nkb ? 0 : nkbi + 1);
        ni = last ? ni : (nkbi == 0 ? ni + 1 : ni);
        const int ic = min(i, len - 1);
        const int src = __builtin_amdgcn_readlane(srcv, ic);
        const int kcg = min(kb * 4 + g, nkc - 1);   // clamped to the tile (B is zero past nq)
        const LT* Au = coup + (p0 + ic) * tile_el + int64_t(kcg) * nq * EPL;
        const LT* Bu = xlo + int64_t(src) * vstride + kb * (4 * ncolp * EPL);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) A[mt] = *reinterpret_cast<const uint4*>(Au + offA[mt]);
        X = *reinterpret_cast<const uint4*>(Bu + offB);
    };
    auto compute = [&](const uint4 (&A)[MT], const uint4& X) {
        const uint4 xr = OPS::re_part(X), xi = OPS::im_part(X);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            acc[mt][0] = OPS::step(A[mt], xr, acc[mt][0]);
            acc[mt][1] = OPS::step(A[mt], xi, acc[mt][1]);
        }
    };
    if (nstep > 0) {
        uint4 A0[MT], A1[MT], X0, X1;
        load(A0, X0);
        for (int j = 0; j < nstep; j += 2) {
            load(A1, X1);
            compute(A0, X0);
            if (j + 1 >= nstep) break;
            load(A0, X0);
            compute(A1, X1);
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            red[wave - 1][mt][0][lane] = acc[mt][0];
            red[wave - 1][mt][1][lane] = acc[mt][1];
        }
    }
    __syncthreads();
    if (wave > 0) return;
    const int c = c0 + li;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        ACC s0 = acc[mt][0], s1 = acc[mt][1];
#pragma unroll
        for (int w = 0; w < NW - 1; ++w) {
            s0 += red[w][mt][0][lane];
            s1 += red[w][mt][1][lane];
        }
        if (c >= ncol) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ar = mt * 16 + OPS::orow(g, r);
            if (ar < nq) part[(ch * nq + ar) * ncol + c] = make_pt<typename OPS::PT>(s0[r], s1[r]);
        }
    }
}

// fp64 coupling without stored tiles: the kernel is evaluated at every node
// pair as the product runs (source node geometry and moments staged in LDS,
// the target node in registers).  Same operator as the stored tiles up to
// rounding; partials and their reduction as in the stored-tile kernels.
template <int NT, int RB>
__global__ __launch_bounds__(NT) void m2l_otf_soft(const double* __restrict__ nodes, const double2* __restrict__ xh,
                                                   const int* __restrict__ far_src_g,
                                                   const int* __restrict__ chunk_tgt,
                                                   const int64_t* __restrict__ chunk_pair,
                                                   const int* __restrict__ chunk_len, int64_t nchunk, int nq, int ncol,
                                                   double kappa, SoftMix mix, double2* __restrict__ part) {
    __shared__ double ys[NT][8];
    __shared__ double2 xs[NT * RB];
    const int64_t ch = blockIdx.x;
    if (ch >= nchunk) return;
    const int c0 = blockIdx.y * RB;
    const int a = threadIdx.x;
    const int64_t p0 = chunk_pair[ch];
    const int len = chunk_len[ch];
    double X[7];
    if (a < nq) {
        const double* T = nodes + (int64_t(chunk_tgt[ch]) * nq + a) * 16;
#pragma unroll
        for (int i = 0; i < 7; ++i) X[i] = T[i];
    }
    double2 acc[RB];
#pragma unroll
    for (int cb = 0; cb < RB; ++cb) acc[cb] = make_double2(0, 0);
    for (int i = 0; i < len; ++i) {
        const int64_t src = far_src_g[p0 + i];
        __syncthreads();
        if (a < nq) {
            const double* Y = nodes + (src * nq + a) * 16;
#pragma unroll
            for (int j = 0; j < 7; ++j) ys[a][j] = Y[j];
        }
        for (int idx = a; idx < nq * RB; idx += NT) {
            const int cb = idx % RB, b = idx / RB;
            xs[idx] = c0 + cb < ncol ? xh[(src * nq + b) * ncol + c0 + cb] : make_double2(0, 0);
        }
        __syncthreads();
        if (a < nq) {
            for (int b = 0; b < nq; ++b) {
                const double2 kv = kernel_soft(X, X + 3, X[6], ys[b], ys[b][6], kappa, mix);
#pragma unroll
                for (int cb = 0; cb < RB; ++cb) acc[cb] = cfma(kv, xs[b * RB + cb], acc[cb]);
            }
        }
    }
    if (a < nq)
#pragma unroll
        for (int cb = 0; cb < RB; ++cb)
            if (c0 + cb < ncol) part[(ch * nq + a) * ncol + c0 + cb] = acc[cb];
}

template <int NT, int RB>
__global__ __launch_bounds__(NT) void m2l_otf_hard(const double* __restrict__ nodes, const double2* __restrict__ xh,
                                                   int64_t kind_stride, const int* __restrict__ far_src_g,
                                                   const int* __restrict__ chunk_tgt,
                                                   const int64_t* __restrict__ chunk_pair,
                                                   const int* __restrict__ chunk_len, int64_t nchunk, int nq, int ncol,
                                                   double kappa, double2* __restrict__ part) {
    __shared__ double ys[NT][3];
    __shared__ double2 sv[7][NT * RB];
    const int64_t ch = blockIdx.x;
    if (ch >= nchunk) return;
    const int c0 = blockIdx.y * RB;
    const int a = threadIdx.x;
    const int64_t p0 = chunk_pair[ch];
    const int len = chunk_len[ch];
    double X[3];
    if (a < nq) {
        const double* T = nodes + (int64_t(chunk_tgt[ch]) * nq + a) * 16;
        X[0] = T[0];
        X[1] = T[1];
        X[2] = T[2];
    }
    double2 rh[4][RB], rg[6][RB];
#pragma unroll
    for (int cb = 0; cb < RB; ++cb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) rh[v][cb] = make_double2(0, 0);
#pragma unroll
        for (int v = 0; v < 6; ++v) rg[v][cb] = make_double2(0, 0);
    }
    for (int i = 0; i < len; ++i) {
        const int64_t src = far_src_g[p0 + i];
        __syncthreads();
        if (a < nq) {
            const double* Y = nodes + (src * nq + a) * 16;
            ys[a][0] = Y[0];
            ys[a][1] = Y[1];
            ys[a][2] = Y[2];
        }
        for (int idx = a; idx < nq * RB; idx += NT) {
            const int cb = idx % RB, b = idx / RB;
            const double* Y = nodes + (src * nq + b) * 16;
            double2 xp = make_double2(0, 0), xu = xp, xv = xp;
            if (c0 + cb < ncol) {
                const int64_t o = (src * nq + b) * ncol + c0 + cb;
                xp = xh[o];
                xu = xh[kind_stride + o];
                xv = xh[2 * kind_stride + o];
            }
            const double yn = Y[0] * Y[3] + Y[1] * Y[4] + Y[2] * Y[5];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sv[c][idx] = cscale(xp, Y[3 + c]);
                sv[4 + c][idx] = make_double2(Y[11 + c] * xu.x - Y[8 + c] * xv.x, Y[11 + c] * xu.y - Y[8 + c] * xv.y);
            }
            sv[3][idx] = cscale(xp, yn);
        }
        __syncthreads();
        if (a < nq) {
            for (int b = 0; b < nq; ++b) {
                double2 G, H;
                kernel_gh(X, ys[b], kappa, G, H);
#pragma unroll
                for (int cb = 0; cb < RB; ++cb) {
                    const int o = b * RB + cb;
                    rh[0][cb] = cfma(H, sv[3][o], rh[0][cb]);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        rh[1 + c][cb] = cfma(H, sv[c][o], rh[1 + c][cb]);
                        rg[c][cb] = cfma(G, sv[c][o], rg[c][cb]);
                        rg[3 + c][cb] = cfma(G, sv[4 + c][o], rg[3 + c][cb]);
                    }
                }
            }
        }
    }
    if (a < nq)
#pragma unroll
        for (int cb = 0; cb < RB; ++cb) {
            if (c0 + cb >= ncol) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) part[((ch * 10 + v) * nq + a) * ncol + c0 + cb] = rh[v][cb];
#pragma unroll
            for (int v = 0; v < 6; ++v) part[((ch * 10 + 4 + v) * nq + a) * ncol + c0 + cb] = rg[v][cb];
        }
}

// fp64 sound-hard coupling without stored tiles for blocks of >= 16 columns
// on the fp64 matrix cores.  Per pair, the G and H values of SLAB source nodes
// at a time are evaluated at every target node into LDS together with the
// slab's source vectors (16 columns, from round_vectors), and the waves
// multiply them as the stored-tile kernel does (H on vectors {3, 0, 1, 2}, G
// on {0, 1, 2, 4, 5, 6}: the vector-path kernel's 10 partials in its order).
// SPLIT: two waves per 16-row tile, one taking the 4 H products and G on
// vector 0, the other G on {1, 2, 4, 5, 6}, so that six row tiles (q = 8)
// give 12 waves, 3 per SIMD, instead of 6 on 4 SIMDs.  Two LDS buffers: each
// thread evaluates the next slab while the matrix cores work through the
// current one; one barrier per slab.  Every output sums the chunk's pairs and
// their source nodes in order, so a column's result does not depend on the
// other columns (nor on SPLIT).  Target rows past nq are not evaluated (zero;
// their outputs are not stored).
template <int NW, int SLAB, bool SPLIT>
__global__ __launch_bounds__(64 * NW * (SPLIT ? 2 : 1)) void m2l_otf_mfma_hard(
    const double* __restrict__ nodes, const double2* __restrict__ xv, int kbp, int ncolp,
    const int* __restrict__ far_src_g, const int* __restrict__ chunk_tgt, const int64_t* __restrict__ chunk_pair,
    const int* __restrict__ chunk_len, int64_t nchunk, int nq, int ncol, double kappa, double2* __restrict__ part) {
    constexpr int R = 16 * NW, NT = 64 * NW * (SPLIT ? 2 : 1), EB = NT / R, KS = SLAB / 4;
    constexpr int NA = SPLIT ? 5 : 10;   // accumulated products per wave
    static_assert(SLAB % 4 == 0 && SLAB % EB == 0, "a slab is whole k blocks and evaluation passes");
    __shared__ double2 gh[2][2][SLAB][R];    // [buffer][G, H][source node in slab][target row]
    __shared__ double2 vs[2][7][SLAB][16];   // [buffer][source vector][source node in slab][column]
    const int64_t ch = xcd_chunk(blockIdx.x, nchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, g = lane >> 4;
    const int rt = SPLIT ? wave >> 1 : wave, half = SPLIT ? wave & 1 : 0;   // row tile, product half
    const int c0 = blockIdx.y * 16;
    const int64_t p0 = chunk_pair[ch];
    const int len = chunk_len[ch];
    const int nkb = (nq + 3) / 4, nsl = (nq + SLAB - 1) / SLAB, nstep = len * nsl;
    // evaluation: fixed target row, source nodes eb0, eb0 + EB, ... of each slab
    const int ea = tid % R, eb0 = tid / R;
    const bool erow = ea < nq;
    double X[3];
    {
        const double* T = nodes + (int64_t(chunk_tgt[ch]) * nq + min(ea, nq - 1)) * 16;
        X[0] = T[0];
        X[1] = T[1];
        X[2] = T[2];
    }
    const int64_t vstride = int64_t(kbp) * ncolp;
    auto stage = [&](int j, int bf) {
        const int i = j / nsl, sl = j % nsl;
        const int64_t src = far_src_g[p0 + i];
        const double* Y = nodes + src * nq * 16;
#pragma unroll
        for (int e = eb0; e < SLAB; e += EB) {
            const int b = sl * SLAB + e;
            double2 G = make_double2(0, 0), H = G;
            if (erow && b < nq) kernel_gh(X, Y + b * 16, kappa, G, H);
            gh[bf][0][e][ea] = G;
            gh[bf][1][e][ea] = H;
        }
        // the source vectors are zero past nq up to kbp; slab nodes past kbp are not read
        for (int e = tid; e < 7 * SLAB * 16; e += NT) {
            const int c = e % 16, b = (e / 16) % SLAB, v = e / (16 * SLAB), bb = sl * SLAB + b;
            vs[bf][v][b][c] = bb < kbp ? xv[(src * 7 + v) * vstride + int64_t(bb) * ncolp + c0 + c] : make_double2(0, 0);
        }
    };
    f64x4 acc[NA][2];
#pragma unroll
    for (int v = 0; v < NA; ++v) acc[v][0] = acc[v][1] = f64x4{0, 0, 0, 0};
    auto product = [&](int o, const uint4& A, const uint4& V) {
        acc[o][0] = MfmaF64::step(A, MfmaF64::re_part(V), acc[o][0]);
        acc[o][1] = MfmaF64::step(A, MfmaF64::im_part(V), acc[o][1]);
    };
    auto consume = [&](int bf, int sl) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            if (sl * KS + ks >= nkb) break;
            const int e = ks * 4 + g;
            auto ld = [&](const double2& x) { return *reinterpret_cast<const uint4*>(&x); };
            const uint4 AG = ld(gh[bf][0][e][rt * 16 + li]);
            if (!SPLIT) {
                const uint4 AH = ld(gh[bf][1][e][rt * 16 + li]);
                uint4 V[7];
#pragma unroll
                for (int v = 0; v < 7; ++v) V[v] = ld(vs[bf][v][e][li]);
                constexpr int hv[4] = {3, 0, 1, 2};
                constexpr int gv[6] = {0, 1, 2, 4, 5, 6};
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) product(jj, AH, V[hv[jj]]);
#pragma unroll
                for (int jj = 0; jj < 6; ++jj) product(4 + jj, AG, V[gv[jj]]);
            } else if (half == 0) {
                const uint4 AH = ld(gh[bf][1][e][rt * 16 + li]);
                const uint4 V0 = ld(vs[bf][0][e][li]), V1 = ld(vs[bf][1][e][li]), V2 = ld(vs[bf][2][e][li]),
                            V3 = ld(vs[bf][3][e][li]);
                product(0, AH, V3);
                product(1, AH, V0);
                product(2, AH, V1);
                product(3, AH, V2);
                product(4, AG, V0);
            } else {
                constexpr int gv[5] = {1, 2, 4, 5, 6};
#pragma unroll
                for (int jj = 0; jj < 5; ++jj) product(jj, AG, ld(vs[bf][gv[jj]][e][li]));
            }
        }
    };
    if (nstep > 0) stage(0, 0);
    __syncthreads();
    for (int j = 0; j < nstep; ++j) {
        if (j + 1 < nstep) stage(j + 1, (j + 1) & 1);
        consume(j & 1, j % nsl);
        __syncthreads();
    }
    // lane holds column li and rows MfmaF64::orow(g, 0..3) of its row tile;
    // this wave's products are the partial vectors v0 .. v0 + NA - 1
    const int c = c0 + li, v0 = SPLIT ? 5 * half : 0;
    if (c >= ncol) return;
#pragma unroll
    for (int v = 0; v < NA; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ar = rt * 16 + MfmaF64::orow(g, r);
            if (ar < nq)
                part[((ch * 10 + v0 + v) * nq + ar) * ncol + c] = make_double2(acc[v][0][r], acc[v][1][r]);
        }
}

// coupling, sound-soft: one workgroup per (chunk of source clusters of one
// target, block of RB columns); lane a owns output row a and RB accumulators
template <int NT, class CT, int RB>
__global__ __launch_bounds__(NT) void m2l_chunks(const CT* __restrict__ coup, const double2* __restrict__ xh,
                                                 const int* __restrict__ far_src_g,
                                                 const int64_t* __restrict__ chunk_pair,
                                                 const int* __restrict__ chunk_len, int64_t nchunk, int nq, int ncol,
                                                 double2* __restrict__ part) {
    __shared__ double2 xs[NT * RB];
    const int64_t ch = blockIdx.x;
    if (ch >= nchunk) return;
    const int c0 = blockIdx.y * RB;
    const int a = threadIdx.x;
    const int64_t p0 = chunk_pair[ch];
    const int len = chunk_len[ch];
    double2 acc[RB];
#pragma unroll
    for (int cb = 0; cb < RB; ++cb) acc[cb] = make_double2(0, 0);
    for (int i = 0; i < len; ++i) {
        const int64_t pr = p0 + i;
        const int64_t src = far_src_g[pr];
        __syncthreads();
        for (int idx = a; idx < nq * RB; idx += NT) {
            const int cb = idx % RB, b = idx / RB;
            xs[idx] = c0 + cb < ncol ? xh[(src * nq + b) * ncol + c0 + cb] : make_double2(0, 0);
        }
        __syncthreads();
        if (a < nq) {
            const CT* K = coup + pr * nq * nq + a;
#pragma unroll 7
            for (int b = 0; b < nq; ++b) {
                const double2 kv = to_d2(K[int64_t(b) * nq]);
#pragma unroll
                for (int cb = 0; cb < RB; ++cb) acc[cb] = cfma(kv, xs[b * RB + cb], acc[cb]);
            }
        }
    }
    if (a < nq)
#pragma unroll
        for (int cb = 0; cb < RB; ++cb)
            if (c0 + cb < ncol) part[(ch * nq + a) * ncol + c0 + cb] = acc[cb];
}

__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long u = __double_as_longlong(v);
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(u & 0xffffffffll), l));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(u >> 32), l));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// coupling, sound-soft, one column, nq <= 64: one wave per chunk.  The source
// moments sit one per lane and reach all lanes by readlane (no LDS, no
// barrier); the next source's moments load while the current tile streams.
// Same products in the same order as m2l_chunks.
__global__ __launch_bounds__(64) void m2l_chunks_wave(const double2* __restrict__ coup,
                                                      const double2* __restrict__ xh,
                                                      const int* __restrict__ far_src_g,
                                                      const int64_t* __restrict__ chunk_pair,
                                                      const int* __restrict__ chunk_len, int64_t nchunk, int nq,
                                                      double2* __restrict__ part) {
    const int64_t ch = blockIdx.x;
    if (ch >= nchunk) return;
    const int a = threadIdx.x;
    const int ac = a < nq ? a : nq - 1;   // idle lanes repeat the last row (never stored)
    const int64_t p0 = chunk_pair[ch];
    const int len = chunk_len[ch];
    double2 acc = make_double2(0, 0);
    double2 xn = xh[int64_t(far_src_g[p0]) * nq + ac];
    for (int i = 0; i < len; ++i) {
        const double2 xv = xn;
        if (i + 1 < len) xn = xh[int64_t(far_src_g[p0 + i + 1]) * nq + ac];
        const double2* K = coup + (p0 + i) * nq * nq + ac;
#pragma unroll 7
        for (int b = 0; b < nq; ++b) {
            const double2 kv = K[int64_t(b) * nq];
            const double2 xb = make_double2(readlane_d(xv.x, b), readlane_d(xv.y, b));
            acc = cfma(kv, xb, acc);
        }
    }
    if (a < nq) part[ch * nq + a] = acc;
}

// Recompression of one fp64 coupling tile K (nq x nq, K(a, b) stored at
// [b*nq + a]: a target node, b source node) by Householder QR with column
// pivoting (the trailing column of largest norm first): K P = Q R.  The
// factorisation stops at the first k with ||R(k:, k:)||_F <= tol ||K||_F, so
// that K ~ U W with U = Q(:, 0:k) and W = R(0:k, :) P^T and
// ||K - U W||_F <= tol ||K||_F.  Reflectors H = I - tau v v^H with v(k) = 1
// (stored below the diagonal), R(k, k) real.  Pass 1 (fac == nullptr) writes
// k; pass 2 repeats the same steps and writes u_k(a) at fac[off + k*nq + a] and
// w_k(b) at fac[off + K*nq + k*nq + b].  One workgroup per tile at a time, the
// tile in LDS (nq <= 64).
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 cconj_mul(double2 a, double2 b) {   // conj(a) b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__global__ __launch_bounds__(256) void tile_rrqr(const double2* __restrict__ coup, int64_t npairs, int nq, double tol,
                                                 int* __restrict__ rank, const int64_t* __restrict__ off,
                                                 double2* __restrict__ fac) {
    __shared__ double2 A[64 * 64];   // column c at A[c*nq + i]
    __shared__ double cn[64];        // squared norms of the trailing columns, rows k..
    __shared__ double2 tau[64];
    __shared__ int perm[64];
    __shared__ double red[256];
    __shared__ double sh_trail;
    __shared__ int sh_piv;
    const int tid = threadIdx.x, n2 = nq * nq;
    const int lane = tid & 63, wave = tid >> 6;
    const int qc = tid >> 2, qr = tid & 3;   // column (offset) and row quarter of this thread in the updates
    for (int64_t p = blockIdx.x; p < npairs; p += gridDim.x) {
        __syncthreads();
        double s = 0;
        for (int i = tid; i < n2; i += 256) {
            const double2 v = coup[p * n2 + i];
            A[i] = v;
            s += v.x * v.x + v.y * v.y;
        }
        if (tid < nq) perm[tid] = tid;
        red[tid] = s;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st) red[tid] += red[tid + st];
            __syncthreads();
        }
        const double total = red[0];
        const int kmax = fac ? rank[p] : nq;
        int k = 0;
        for (; k < nq; ++k) {
            // squared norms of the trailing columns over rows k..nq-1
            if (tid < nq) {
                double c2 = 0;
                if (tid >= k)
                    for (int i = k; i < nq; ++i) {
                        const double2 v = A[tid * nq + i];
                        c2 += v.x * v.x + v.y * v.y;
                    }
                cn[tid] = c2;
            }
            __syncthreads();
            if (wave == 0) {
                double sum = lane < nq && lane >= k ? cn[lane] : 0.0;
                double mx = lane < nq && lane >= k ? cn[lane] : -1.0;
                int mi = lane;
                for (int o = 32; o >= 1; o >>= 1) {
                    sum += __shfl_xor(sum, o, 64);
                    const double om = __shfl_xor(mx, o, 64);
                    const int oi = __shfl_xor(mi, o, 64);
                    if (om > mx || (om == mx && oi < mi)) {
                        mx = om;
                        mi = oi;
                    }
                }
                if (lane == 0) {
                    sh_trail = sum;
                    sh_piv = mi;
                }
            }
            __syncthreads();
            if (k >= kmax || !(sh_trail > tol * tol * total)) break;
            const int pv = sh_piv;
            if (pv != k) {
                for (int i = tid; i < nq; i += 256) {
                    const double2 t = A[k * nq + i];
                    A[k * nq + i] = A[pv * nq + i];
                    A[pv * nq + i] = t;
                }
                if (tid == 0) {
                    const int t = perm[k];
                    perm[k] = perm[pv];
                    perm[pv] = t;
                }
            }
            __syncthreads();
            // reflector of column k, rows k..nq-1
            if (wave == 0) {
                const double2 x = lane > k && lane < nq ? A[k * nq + lane] : make_double2(0, 0);
                double xn2 = x.x * x.x + x.y * x.y;
                for (int o = 32; o >= 1; o >>= 1) xn2 += __shfl_xor(xn2, o, 64);
                const double2 al = A[k * nq + k];
                double2 t = make_double2(0, 0);
                if (xn2 > 0 || al.y != 0) {
                    const double beta = -copysign(sqrt(al.x * al.x + al.y * al.y + xn2), al.x);
                    t = make_double2((beta - al.x) / beta, -al.y / beta);
                    const double2 sc = cdiv(make_double2(1.0, 0.0), make_double2(al.x - beta, al.y));
                    if (lane > k && lane < nq) A[k * nq + lane] = cmul(x, sc);
                    if (lane == 0) A[k * nq + k] = make_double2(beta, 0.0);
                }
                if (lane == 0) tau[k] = t;
            }
            __syncthreads();
            // A(k:, c) -= conj(tau) v (v^H A(k:, c)) for the columns c > k
            const double2 tk = tau[k];
            const int c = k + 1 + qc;
            double2 dot = make_double2(0, 0);
            if (c < nq)
                for (int i = k + qr; i < nq; i += 4) {
                    const double2 v = i == k ? make_double2(1.0, 0.0) : A[k * nq + i];
                    dot = cadd(dot, cconj_mul(v, A[c * nq + i]));
                }
            dot.x += __shfl_xor(dot.x, 1, 64);
            dot.y += __shfl_xor(dot.y, 1, 64);
            dot.x += __shfl_xor(dot.x, 2, 64);
            dot.y += __shfl_xor(dot.y, 2, 64);
            const double2 wv = cmul(make_double2(tk.x, -tk.y), dot);
            if (c < nq)
                for (int i = k + qr; i < nq; i += 4) {
                    const double2 v = i == k ? make_double2(1.0, 0.0) : A[k * nq + i];
                    const double2 d = cmul(v, wv);
                    A[c * nq + i] = make_double2(A[c * nq + i].x - d.x, A[c * nq + i].y - d.y);
                }
            __syncthreads();
        }
        const int K = k;
        if (!fac) {
            if (tid == 0) rank[p] = K;
            continue;
        }
        const int64_t o = off[p];
        // W = R(0:K, :) P^T
        for (int e = tid; e < nq * K; e += 256) {
            const int j = e / K, kk = e % K;
            fac[o + int64_t(K) * nq + int64_t(kk) * nq + perm[j]] = kk <= j ? A[j * nq + kk] : make_double2(0, 0);
        }
        __syncthreads();
        // Q(:, 0:K) in place, from the last reflector to the first: columns i+1..K-1
        // already hold Q's columns when H_i is applied to them
        for (int i = K - 1; i >= 0; --i) {
            const double2 ti = tau[i];
            const int c = i + 1 + qc;
            double2 dot = make_double2(0, 0);
            if (c < K)
                for (int r = i + qr; r < nq; r += 4) {
                    const double2 v = r == i ? make_double2(1.0, 0.0) : A[i * nq + r];
                    dot = cadd(dot, cconj_mul(v, A[c * nq + r]));
                }
            dot.x += __shfl_xor(dot.x, 1, 64);
            dot.y += __shfl_xor(dot.y, 1, 64);
            dot.x += __shfl_xor(dot.x, 2, 64);
            dot.y += __shfl_xor(dot.y, 2, 64);
            const double2 wv = cmul(ti, dot);
            if (c < K)
                for (int r = i + qr; r < nq; r += 4) {
                    const double2 v = r == i ? make_double2(1.0, 0.0) : A[i * nq + r];
                    const double2 d = cmul(v, wv);
                    A[c * nq + r] = make_double2(A[c * nq + r].x - d.x, A[c * nq + r].y - d.y);
                }
            __syncthreads();
            // column i of Q: (1 - tau) at row i, -tau v below, zero above
            for (int r = tid; r < nq; r += 256) {
                const double2 v = A[i * nq + r];
                A[i * nq + r] = r < i ? make_double2(0, 0)
                                      : r == i ? make_double2(1.0 - ti.x, -ti.y)
                                               : make_double2(-(ti.x * v.x - ti.y * v.y), -(ti.x * v.y + ti.y * v.x));
            }
            __syncthreads();
        }
        for (int e = tid; e < nq * K; e += 256) fac[o + e] = A[e];
    }
}

// operator data streamed once per product: non-temporal loads leave the
// caches to the vectors the product reuses
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_nt(const double2* p) {
    const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
    return make_double2(v.x, v.y);
}

constexpr int LR_WAVES = 8;
// coupling, sound-soft, one column, from the recompressed tiles: one
// workgroup of NW waves per chunk (up to 8 pairs of one target), wave w taking
// the pairs w, w + NW, ...  For each pair and group of 8 terms k: the rows
// w_k(.) and u_k(.) are read full width (lane = node), lane b forms
// w_k(b) x(b) with the source moment it holds, the 8 sums over b are reduced
// together (three halving exchanges leave lane L with term k = 4 L5 + 2 L4 +
// L3 of the group, L5..L3 its bits 5..3, three more complete the sum), and
// y(a) += u_k(a) t_k for the group's terms below the rank.  Rows past the rank
// are read at the last row (their sums are never used); lanes past nq hold a
// zero moment.  The waves' sums meet in LDS in wave order.
__device__ __forceinline__ double2 shfl_xor_c(double2 v, int m) {
    return make_double2(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}
template <int NW>
__global__ __launch_bounds__(64 * NW) void m2l_chunks_lowrank(const double2* __restrict__ fac,
                                                              const int* __restrict__ rank,
                                                              const int64_t* __restrict__ off,
                                                              const double2* __restrict__ xh,
                                                              const int* __restrict__ far_src_g,
                                                              const int64_t* __restrict__ chunk_pair,
                                                              const int* __restrict__ chunk_len, int64_t nchunk,
                                                              int nq, double2* __restrict__ part) {
    constexpr int PW = (M2L_CHUNK + NW - 1) / NW;   // pairs per wave
    __shared__ double2 red[NW > 1 ? NW - 1 : 1][64];
    const int64_t ch = blockIdx.x;
    if (ch >= nchunk) return;
    const int a = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ac = a < nq ? a : nq - 1;
    const int64_t p0 = chunk_pair[ch];
    const int len = chunk_len[ch];
    const int rk = a < len ? rank[p0 + a] : 0;
    const int64_t of = a < len ? off[p0 + a] : 0;
    const int sr = a < len ? far_src_g[p0 + a] : 0;
    const bool hi5 = a & 32, hi4 = a & 16, hi3 = a & 8;
    double2 acc = make_double2(0, 0);
#pragma unroll
    for (int j = 0; j < PW; ++j) {
        const int i = wave + NW * j;   // pair of the chunk
        const int K = i < M2L_CHUNK ? __builtin_amdgcn_readlane(rk, i) : 0;
        if (K == 0) continue;   // past the chunk or rank 0 (uniform)
        const int64_t o = (int64_t(__builtin_amdgcn_readlane(int(of >> 32), i)) << 32) |
                          unsigned(__builtin_amdgcn_readlane(int(of & 0xffffffff), i));
        const double2 xv = a < nq ? xh[int64_t(__builtin_amdgcn_readlane(sr, i)) * nq + a] : make_double2(0, 0);
        const double2* U = fac + o;
        const double2* Wr = fac + o + int64_t(K) * nq;
        for (int k0 = 0; k0 < K; k0 += 8) {
            double2 p[8], u[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int k = min(k0 + r, K - 1);
                const double2 wv = Wr[int64_t(k) * nq + ac];
                u[r] = U[int64_t(k) * nq + ac];
                p[r] = cmul(wv, xv);
            }
            double2 q4[4], q2[2], q1;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double2 keep = hi5 ? p[4 + r] : p[r], give = hi5 ? p[r] : p[4 + r];
                q4[r] = cadd(keep, shfl_xor_c(give, 32));
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const double2 keep = hi4 ? q4[2 + r] : q4[r], give = hi4 ? q4[r] : q4[2 + r];
                q2[r] = cadd(keep, shfl_xor_c(give, 16));
            }
            {
                const double2 keep = hi3 ? q2[1] : q2[0], give = hi3 ? q2[0] : q2[1];
                q1 = cadd(keep, shfl_xor_c(give, 8));
            }
            q1 = cadd(q1, shfl_xor_c(q1, 4));
            q1 = cadd(q1, shfl_xor_c(q1, 2));
            q1 = cadd(q1, shfl_xor_c(q1, 1));
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                if (k0 + r >= K) break;   // uniform
                const int src_lane = ((r & 4) ? 32 : 0) + ((r & 2) ? 16 : 0) + ((r & 1) ? 8 : 0);
                const double2 tk = make_double2(readlane_d(q1.x, src_lane), readlane_d(q1.y, src_lane));
                acc = cfma(u[r], tk, acc);
            }
        }
    }
    if (NW > 1) {
        if (wave > 0) red[wave - 1][a] = acc;
        __syncthreads();
        if (wave > 0) return;
#pragma unroll
        for (int w = 0; w < NW - 1; ++w) acc = cadd(acc, red[w][a]);
    }
    if (a < nq) part[ch * nq + a] = acc;
}

// coupling, sound-hard: per source the 7 node-scaled moment vectors
//   n~_c xp (c = 0..2), (y.n~) xp, v_c = F_v,c xu - F_u,c xv
// are formed in LDS; H acts on {(y.n~) xp, n~_c xp}, G on {n~_c xp, v_c}:
// 10 partial vectors per chunk and column.
template <int NT, class CT, int RB>
__global__ __launch_bounds__(NT) void m2l_hard_chunks(const CT* __restrict__ coup, const double2* __restrict__ xh,
                                                      int64_t kind_stride, const double* __restrict__ nodes,
                                                      const int* __restrict__ far_src_g,
                                                      const int64_t* __restrict__ chunk_pair,
                                                      const int* __restrict__ chunk_len, int64_t nchunk, int nq,
                                                      int ncol, double2* __restrict__ part) {
    __shared__ double2 sv[7][NT * RB];
    const int64_t ch = blockIdx.x;
    if (ch >= nchunk) return;
    const int c0 = blockIdx.y * RB;
    const int a = threadIdx.x;
    const int64_t p0 = chunk_pair[ch];
    const int len = chunk_len[ch];
    double2 rh[4][RB], rg[6][RB];
#pragma unroll
    for (int cb = 0; cb < RB; ++cb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) rh[v][cb] = make_double2(0, 0);
#pragma unroll
        for (int v = 0; v < 6; ++v) rg[v][cb] = make_double2(0, 0);
    }
    for (int i = 0; i < len; ++i) {
        const int64_t pr = p0 + i;
        const int64_t src = far_src_g[pr];
        __syncthreads();
        for (int idx = a; idx < nq * RB; idx += NT) {
            const int cb = idx % RB, b = idx / RB;
            const double* Y = nodes + (src * nq + b) * 16;
            double2 xp = make_double2(0, 0), xu = xp, xv = xp;
            if (c0 + cb < ncol) {
                const int64_t o = (src * nq + b) * ncol + c0 + cb;
                xp = xh[o];
                xu = xh[kind_stride + o];
                xv = xh[2 * kind_stride + o];
            }
            const double yn = Y[0] * Y[3] + Y[1] * Y[4] + Y[2] * Y[5];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sv[c][idx] = cscale(xp, Y[3 + c]);
                sv[4 + c][idx] = make_double2(Y[11 + c] * xu.x - Y[8 + c] * xv.x, Y[11 + c] * xu.y - Y[8 + c] * xv.y);
            }
            sv[3][idx] = cscale(xp, yn);
        }
        __syncthreads();
        if (a < nq) {
            const CT* K = coup + pr * nq * nq * 2 + a;
            for (int b = 0; b < nq; ++b) {
                const double2 G = to_d2(K[int64_t(b) * nq]), H = to_d2(K[int64_t(nq + b) * nq]);
#pragma unroll
                for (int cb = 0; cb < RB; ++cb) {
                    const int o = b * RB + cb;
                    rh[0][cb] = cfma(H, sv[3][o], rh[0][cb]);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        rh[1 + c][cb] = cfma(H, sv[c][o], rh[1 + c][cb]);
                        rg[c][cb] = cfma(G, sv[c][o], rg[c][cb]);
                        rg[3 + c][cb] = cfma(G, sv[4 + c][o], rg[3 + c][cb]);
                    }
                }
            }
        }
    }
    if (a < nq)
#pragma unroll
        for (int cb = 0; cb < RB; ++cb) {
            if (c0 + cb >= ncol) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) part[((ch * 10 + v) * nq + a) * ncol + c0 + cb] = rh[v][cb];
#pragma unroll
            for (int v = 0; v < 6; ++v) part[((ch * 10 + 4 + v) * nq + a) * ncol + c0 + cb] = rg[v][cb];
        }
}

// target-side factors of the sound-hard coupling:
//   y_p = -a R0 + a sum_c x_c R_c + i eta kappa^2 sum_c n~_c S_c
//   y_u = -i eta sum_c F_v,c T_c,   y_v = +i eta sum_c F_u,c T_c
// from raw[cluster][10][nq][C] = (R0, R_0..2, S_0..2, T_0..2)
__global__ void m2l_finalize_hard(const double2* raw, const double* nodes, int64_t nclusters, int nq, double kappa,
                                  HardMix hmix, int64_t kind_stride, int ncol, double2* yh) {
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= nclusters * nq * ncol) return;
    const int r = int(gid % ncol);
    const int64_t t = gid / ncol;
    const int64_t c = t / nq;
    const int a = int(t % nq);
    const double* X = nodes + t * 16;
    const double2* rw = raw + (c * 10 * nq + a) * ncol + r;
    const int64_t vs = int64_t(nq) * ncol;
    double2 yp = cscale(rw[0], -X[6]);
    double2 su = make_double2(0, 0), sv = make_double2(0, 0), sn = make_double2(0, 0);
    for (int cc = 0; cc < 3; ++cc) {
        yp = cadd(yp, cscale(rw[(1 + cc) * vs], X[6] * X[cc]));
        sn = cadd(sn, cscale(rw[(4 + cc) * vs], X[3 + cc]));
        su = cadd(su, cscale(rw[(7 + cc) * vs], X[11 + cc]));
        sv = cadd(sv, cscale(rw[(7 + cc) * vs], X[8 + cc]));
    }
    // yp is the -K part: ck K = -ck yp; W: -kappa^2 sn (normal part), su - sv (curl part)
    const double2 mck = make_double2(-hmix.ck.x, -hmix.ck.y);
    yh[gid] = cadd(cmul(mck, yp), cscale(cmul(hmix.cw, sn), -kappa * kappa));
    yh[kind_stride + gid] = cmul(hmix.cw, su);
    yh[2 * kind_stride + gid] = cscale(cmul(hmix.cw, sv), -1.0);
}

// sum over the target's chunks (fixed order), zero if none:
// [chunk][per] -> [cluster][per], per = nvec * nq * ncol
template <class PT>
__global__ void m2l_reduce(const PT* part, const int* tgt_chunk_ptr, int64_t nclusters, int64_t per, double2* yh) {
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= nclusters * per) return;
    const int64_t c = gid / per;
    const int64_t va = gid % per;
    double2 s = make_double2(0, 0);
    for (int ch = tgt_chunk_ptr[c]; ch < tgt_chunk_ptr[c + 1]; ++ch) s = cadd(s, to_d2(part[int64_t(ch) * per + va]));
    yh[gid] = s;
}

constexpr int SPMV_U1 = 4;   // row strides in flight per lane of the one-column near product

// y[r][row] = sum_j val x[r][col] (+ far part mapped to the solution space); one
// wave per row, lanes stride over the row, butterfly reduction (fixed order).
// Columns come from the row's group list (rows with the same leaves share one),
// so the index reads mostly hit the caches and HBM streams the values alone
// (non-temporal loads: the values are read once per product, x and the
// column lists stay in the caches).
// (RB columns per pass; consecutive nonzeros of a row mostly have consecutive
// columns, so the lanes' x reads coalesce.  Each column's operations and
// their order do not depend on RB.  On the m = 5 sphere with 16 columns,
// 4 per pass ran in 0.15 ms, 8 in 0.19 ms and 16 in 0.24 ms.)
template <int RB>
__global__ __launch_bounds__(256) void spmv_combine(const int64_t* __restrict__ row_ptr,
                                                    const int64_t* __restrict__ row_coff,
                                                    const int* __restrict__ col,
                                                    const double2* __restrict__ val,
                                                    const double2* __restrict__ x, int64_t nrows,
                                                    FarLeaves F, const int* __restrict__ s0_ptr,
                                                    const int* __restrict__ s0_reps, int use_near, int ncol,
                                                    double2* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    // consecutive rows on the same XCD: rows of one group read its column
    // list from that XCD's L2 instead of once per XCD
    const int64_t row = xcd_chunk(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= nrows) return;
    const int64_t b = row_ptr[row], e = row_ptr[row + 1];
    const int64_t cbase = row_coff[row] - b;   // the row's shared column list, indexed like its values
    for (int c0 = 0; c0 < ncol; c0 += RB) {
        double2 acc[RB];
#pragma unroll
        for (int cb = 0; cb < RB; ++cb) acc[cb] = make_double2(0, 0);
        if (use_near) {
            // one column: U strides of the row per trip, their loads issued
            // before the first product (more bytes in flight per wave); the
            // products still enter acc in idx order
            constexpr int U = RB == 1 ? SPMV_U1 : 1;
            int64_t idx = b + lane;
            for (; idx + (U - 1) * 64 < e; idx += U * 64) {
                double2 v[U];
                int cc[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    v[u] = ld_nt(val + idx + u * 64);
                    cc[u] = col[cbase + idx + u * 64];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int cb = 0; cb < RB; ++cb)
                        if (c0 + cb < ncol) acc[cb] = cfma(v[u], x[int64_t(c0 + cb) * nrows + cc[u]], acc[cb]);
            }
            for (; idx < e; idx += 64) {
                const double2 v = ld_nt(val + idx);
                const int64_t cc = col[cbase + idx];
#pragma unroll
                for (int cb = 0; cb < RB; ++cb)
                    if (c0 + cb < ncol) acc[cb] = cfma(v, x[int64_t(c0 + cb) * nrows + cc], acc[cb]);
            }
        }
#pragma unroll
        for (int cb = 0; cb < RB; ++cb)
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                acc[cb].x += __shfl_xor(acc[cb].x, off, 64);
                acc[cb].y += __shfl_xor(acc[cb].y, off, 64);
            }
        if (lane == 0) {
#pragma unroll
            for (int cb = 0; cb < RB; ++cb) {
                const int r = c0 + cb;
                if (r >= ncol) continue;
                double2 a = acc[cb];
                if (F.leafbuf) {
                    if (s0_ptr) {
                        for (int q = s0_ptr[row]; q < s0_ptr[row + 1]; ++q) a = cadd(a, far_value(F, s0_reps[q], r));
                    } else {
                        a = cadd(a, far_value(F, row, r));
                    }
                }
                y[int64_t(r) * nrows + row] = a;
            }
        }
    }
}

// The one-column near product by groups: a workgroup takes up to
// NEAR_GROUP_ROWS rows of one group, gathers the group's x entries into LDS in
// list order (every row of the group has exactly the group's columns, entry j
// of a row belonging to list entry j), and then each wave forms one row's sum
// against LDS: no column index and no x gather per nonzero.  The lanes, trips
// and butterfly are those of spmv_combine<1>, with the same x values, so the
// rows equal spmv_combine's bitwise.
template <int NWV>
__global__ __launch_bounds__(64 * NWV) void spmv_groups(const NearGroupWG* __restrict__ wgs,
                                                        const int* __restrict__ grp_rows,
                                                        const int64_t* __restrict__ row_ptr,
                                                        const int* __restrict__ col,
                                                        const double2* __restrict__ val,
                                                        const double2* __restrict__ x,
                                                        FarLeaves F, const int* __restrict__ s0_ptr,
                                                        const int* __restrict__ s0_reps, double2* __restrict__ y) {
    extern __shared__ double2 xs[];
    // consecutive workgroups (the same or neighbouring groups) on one XCD
    const NearGroupWG W = wgs[xcd_chunk(blockIdx.x, gridDim.x)];
    for (int j = threadIdx.x; j < W.list_len; j += 64 * NWV) xs[j] = x[col[W.list_off + j]];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave >= W.nrows) return;
    const int row = grp_rows[W.row0 + wave];
    const double2* v0 = val + row_ptr[row];
    const int len = W.list_len;
    constexpr int U = SPMV_U1;
    double2 acc = make_double2(0, 0);
    int j = lane;
    for (; j + (U - 1) * 64 < len; j += U * 64) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld_nt(v0 + j + u * 64);
#pragma unroll
        for (int u = 0; u < U; ++u) acc = cfma(v[u], xs[j + u * 64], acc);
    }
    for (; j < len; j += 64) acc = cfma(ld_nt(v0 + j), xs[j], acc);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        acc.x += __shfl_xor(acc.x, off, 64);
        acc.y += __shfl_xor(acc.y, off, 64);
    }
    if (lane == 0) {
        if (F.leafbuf) {
            if (s0_ptr) {
                for (int q = s0_ptr[row]; q < s0_ptr[row + 1]; ++q) acc = cadd(acc, far_value(F, s0_reps[q], 0));
            } else {
                acc = cadd(acc, far_value(F, row, 0));
            }
        }
        y[row] = acc;
    }
}

// fp32 tile layout of the near field: tile t holds its rows' values as
// [k block][row][8] over the tile's column list (zero where the row has no
// entry and past the list's end), rounded (RNE) from the fp64 CSR values.
// One thread per row walks the tile's list and the row's (both sorted; the
// tile's list holds the row's).
__global__ void near_tile_values(const NearTile* __restrict__ tiles, const int* __restrict__ tcol,
                                 const int64_t* __restrict__ row_ptr, const int* __restrict__ col,
                                 const double2* __restrict__ val, float2* __restrict__ vt) {
    const NearTile& T = tiles[blockIdx.x];
    const int i = threadIdx.x;
    if (i >= T.nrows) return;
    const int nr = T.nrows, nc = T.ncols;
    const int* tc = tcol + T.col_off;
    const int r = T.rows[i];
    int64_t q = row_ptr[r];
    const int64_t qe = row_ptr[r + 1];
    const int nk = (nc + NEAR_TILE_K - 1) / NEAR_TILE_K * NEAR_TILE_K;
    for (int k = 0; k < nk; ++k) {
        float2 v = make_float2(0.f, 0.f);
        if (k < nc && q < qe && col[q] == tc[k]) {
            const double2 d = val[q++];
            v = make_float2(float(d.x), float(d.y));
        }
        vt[T.val_off + (int64_t(k / NEAR_TILE_K) * nr + i) * NEAR_TILE_K + k % NEAR_TILE_K] = v;
    }
}

// x^T for the tile product: xt[b][row][16] = x[16 b + c][row] rounded to fp32
// (zero for columns past ncol)
__global__ void round_columns_t(const double2* __restrict__ x, int64_t nrows, int ncol, int ncb,
                                float2* __restrict__ xt) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(ncb) * nrows * 16) return;
    const int c = int(i / (nrows * 16)) * 16 + int(i % 16);
    const int64_t row = (i / 16) % nrows;
    float2 v = make_float2(0.f, 0.f);
    if (c < ncol) {
        const double2 d = x[int64_t(c) * nrows + row];
        v = make_float2(float(d.x), float(d.y));
    }
    xt[i] = v;
}

// Near product of the reduced-precision operator (inner matvecs of the bf16
// refinement) on the matrix cores: for one tile of rows and 16 columns,
// Y = V X with the tile values V over the tile's column list (rows past nrows
// are zero) as the A operand and the fp32 columns gathered by that list as
// the B operand, fp32 products and sums.  The 16 waves take every 16th k
// block of 8 columns and meet in LDS in wave order (fixed); the far part is
// added and stored in fp64.  Each output column depends only on its own input column,
// in an order fixed by the tile, so blocks of any width give bitwise the
// results of one column at a time.
constexpr int NEAR_TILE_CHUNK = 2048;   // column indices staged in LDS at a time (multiple of 32)
constexpr int NEAR_TILE_WAVES = 16;
__global__ __launch_bounds__(64 * NEAR_TILE_WAVES) void near_tiles_mfma(const NearTile* __restrict__ tiles, int64_t ntile,
                                                       const int* __restrict__ tcol, const float2* __restrict__ vt,
                                                       const float2* __restrict__ xt, int64_t nrows,
                                                       FarLeaves F, const int* __restrict__ s0_ptr,
                                                       const int* __restrict__ s0_reps, int use_near, int ncol,
                                                       double2* __restrict__ y) {
    constexpr int NW = NEAR_TILE_WAVES;
    __shared__ f32x4 red[NW - 1][2][64];
    __shared__ int cidx[NEAR_TILE_CHUNK];
    const int64_t t = xcd_chunk(blockIdx.x, ntile);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    const NearTile& T = tiles[t];
    const int nr = T.nrows, nc = T.ncols;
    const int nkb = (nc + NEAR_TILE_K - 1) / NEAR_TILE_K;
    const float2* xb = xt + int64_t(blockIdx.y) * nrows * 16 + li;
    const int* cl = tcol + T.col_off;
    const float2* va = vt + T.val_off + li * NEAR_TILE_K + 2 * g;
    const int64_t kbstride = int64_t(nr) * NEAR_TILE_K;
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    auto load = [&](int kb, int kl, uint4& A, uint4& X) {
        A = make_uint4(0u, 0u, 0u, 0u);
        if (li < nr) A = *reinterpret_cast<const uint4*>(va + kb * kbstride);
        const float2 xa = xb[int64_t(cidx[kl + 2 * g]) * 16];
        const float2 xc = xb[int64_t(cidx[kl + 2 * g + 1]) * 16];
        X = make_uint4(__float_as_uint(xa.x), __float_as_uint(xa.y), __float_as_uint(xc.x), __float_as_uint(xc.y));
    };
    auto compute = [&](const uint4& A, const uint4& X) {
        acc0 = MfmaF32::step(A, MfmaF32::re_part(X), acc0);
        acc1 = MfmaF32::step(A, MfmaF32::im_part(X), acc1);
    };
    if (use_near) {
        // chunks of columns: indices to LDS (columns past the list repeat its last
        // one; their values are zero), then each wave's k blocks kb = wave mod 16
        // in increasing order, two loads in flight (16 waves per tile: a few
        // hundred tiles must keep the chip's loads in flight)
        for (int k0 = 0; k0 < nkb * NEAR_TILE_K; k0 += NEAR_TILE_CHUNK) {
            __syncthreads();
            for (int i = threadIdx.x; i < NEAR_TILE_CHUNK; i += blockDim.x) cidx[i] = cl[min(k0 + i, nc - 1)];
            __syncthreads();
            const int kb0 = k0 / NEAR_TILE_K, kb1 = min(nkb, kb0 + NEAR_TILE_CHUNK / NEAR_TILE_K);
            int kb = kb0 + wave;
            for (; kb + NW < kb1; kb += 2 * NW) {
                uint4 A0, X0, A1, X1;
                load(kb, (kb - kb0) * NEAR_TILE_K, A0, X0);
                load(kb + NW, (kb + NW - kb0) * NEAR_TILE_K, A1, X1);
                compute(A0, X0);
                compute(A1, X1);
            }
            if (kb < kb1) {
                uint4 A0, X0;
                load(kb, (kb - kb0) * NEAR_TILE_K, A0, X0);
                compute(A0, X0);
            }
        }
    }
    if (wave > 0) {
        red[wave - 1][0][lane] = acc0;
        red[wave - 1][1][lane] = acc1;
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 0; w < NW - 1; ++w) {
        acc0 += red[w][0][lane];
        acc1 += red[w][1][lane];
    }
    const int c = blockIdx.y * 16 + li;
    if (c >= ncol) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = MfmaF32::orow(g, r);
        if (i >= nr) continue;
        const int row = T.rows[i];
        double2 a = make_double2(double(acc0[r]), double(acc1[r]));
        if (F.leafbuf) {
            if (s0_ptr) {
                for (int q = s0_ptr[row]; q < s0_ptr[row + 1]; ++q) a = cadd(a, far_value(F, s0_reps[q], c));
            } else {
                a = cadd(a, far_value(F, row, c));
            }
        }
        y[int64_t(c) * nrows + row] = a;
    }
}

// fp64 tile layout of the near field for blocks of >= 16 columns of fp64
// operators: tile t holds its rows' values as [k block of 4][row][4] over the
// tile's column list, zero where a row has no entry (the same tiles and column
// lists as the fp32 layout, at the same offsets: a tile's fp64 region is no
// longer than its fp32 one).
__global__ void near_tile_values64(const NearTile* __restrict__ tiles, const int* __restrict__ tcol,
                                   const int64_t* __restrict__ row_ptr, const int* __restrict__ col,
                                   const double2* __restrict__ val, double2* __restrict__ vt) {
    const NearTile& T = tiles[blockIdx.x];
    const int i = threadIdx.x;
    if (i >= T.nrows) return;
    const int nr = T.nrows, nc = T.ncols;
    const int* tc = tcol + T.col_off;
    const int r = T.rows[i];
    int64_t q = row_ptr[r];
    const int64_t qe = row_ptr[r + 1];
    const int nk = (nc + MfmaF64::KB - 1) / MfmaF64::KB * MfmaF64::KB;
    for (int k = 0; k < nk; ++k) {
        double2 v = make_double2(0.0, 0.0);
        if (k < nc && q < qe && col[q] == tc[k]) v = val[q++];
        vt[T.val_off + (int64_t(k / MfmaF64::KB) * nr + i) * MfmaF64::KB + k % MfmaF64::KB] = v;
    }
}

// x^T for the fp64 tile product: xt[b][row][16] = x[16 b + c][row] (zero for
// columns past ncol)
__global__ void columns_t64(const double2* __restrict__ x, int64_t nrows, int ncol, int ncb, double2* __restrict__ xt) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(ncb) * nrows * 16) return;
    const int c = int(i / (nrows * 16)) * 16 + int(i % 16);
    const int64_t row = (i / 16) % nrows;
    xt[i] = c < ncol ? x[int64_t(c) * nrows + row] : make_double2(0.0, 0.0);
}

// Near product of fp64 operators for blocks of >= 16 columns on the fp64
// matrix cores: per tile and NC tiles of 16 columns, Y = V X with the fp64 tile
// values as the A operand (16 rows; rows past nrows read row 0, their outputs
// are not stored) and the columns gathered through the tile's column list as
// the B operand, so every tile value read serves 16 NC columns.  The waves take
// every NW-th k block of 4 columns in increasing order and meet in LDS in wave
// order; each output column depends only on its own input column in an order
// fixed by the tile, so every block of >= 16 columns gives bitwise the same
// column results (which differ from the one-column CSR product by rounding:
// another summation order).
constexpr int NEAR64_WAVES = 8;
template <int NC>
__global__ __launch_bounds__(64 * NEAR64_WAVES) void near_tiles_mfma64(
    const NearTile* __restrict__ tiles, int64_t ntile, const int* __restrict__ tcol, const double2* __restrict__ vt,
    const double2* __restrict__ xt, int64_t nrows, FarLeaves F,
    const int* __restrict__ s0_ptr, const int* __restrict__ s0_reps, int use_near, int ncol,
    double2* __restrict__ y) {
    constexpr int NW = NEAR64_WAVES, KB = MfmaF64::KB;
    __shared__ f64x4 red[NW - 1][2][64];
    __shared__ int cidx[NEAR_TILE_CHUNK];
    const int64_t t = xcd_chunk(blockIdx.x, ntile);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, g = lane >> 4;
    const NearTile& T = tiles[t];
    const int nr = T.nrows, nc = T.ncols;
    const int nkb = (nc + KB - 1) / KB;
    // column tile j of this workgroup: block (NC blockIdx.y + j) of the
    // transposed columns [block][row][16]
    const double2* xb = xt + int64_t(blockIdx.y) * NC * nrows * 16 + li;
    const int* cl = tcol + T.col_off;
    const int ra = li < nr ? li : 0;
    const double2* va = vt + T.val_off + ra * KB + g;
    const int64_t kbstride = int64_t(nr) * KB;
    f64x4 acc[NC][2];
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j][0] = acc[j][1] = f64x4{0.0, 0.0, 0.0, 0.0};
    auto load = [&](int kb, int kl, uint4& A, uint4 (&X)[NC]) {
        A = *reinterpret_cast<const uint4*>(va + kb * kbstride);
        const int64_t o = int64_t(cidx[kl + g]) * 16;
#pragma unroll
        for (int j = 0; j < NC; ++j) X[j] = *reinterpret_cast<const uint4*>(xb + int64_t(j) * nrows * 16 + o);
    };
    auto compute = [&](const uint4& A, const uint4 (&X)[NC]) {
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            acc[j][0] = MfmaF64::step(A, MfmaF64::re_part(X[j]), acc[j][0]);
            acc[j][1] = MfmaF64::step(A, MfmaF64::im_part(X[j]), acc[j][1]);
        }
    };
    if (use_near) {
        // chunks of columns: indices to LDS (past the list: its last column, whose
        // tile values are zero there), then each wave's k blocks kb = wave mod NW
        // in increasing order, two loads in flight
        for (int k0 = 0; k0 < nkb * KB; k0 += NEAR_TILE_CHUNK) {
            __syncthreads();
            for (int i = threadIdx.x; i < NEAR_TILE_CHUNK; i += blockDim.x) cidx[i] = cl[min(k0 + i, nc - 1)];
            __syncthreads();
            const int kb0 = k0 / KB, kb1 = min(nkb, kb0 + NEAR_TILE_CHUNK / KB);
            int kb = kb0 + wave;
            for (; kb + NW < kb1; kb += 2 * NW) {
                uint4 A0, X0[NC], A1, X1[NC];
                load(kb, (kb - kb0) * KB, A0, X0);
                load(kb + NW, (kb + NW - kb0) * KB, A1, X1);
                compute(A0, X0);
                compute(A1, X1);
            }
            if (kb < kb1) {
                uint4 A0, X0[NC];
                load(kb, (kb - kb0) * KB, A0, X0);
                compute(A0, X0);
            }
        }
    }
    // the waves' sums meet in LDS in wave order, one column tile at a time
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        __syncthreads();
        if (wave > 0) {
            red[wave - 1][0][lane] = acc[j][0];
            red[wave - 1][1][lane] = acc[j][1];
        }
        __syncthreads();
        if (wave == 0) {
            f64x4 s0 = acc[j][0], s1 = acc[j][1];
#pragma unroll
            for (int w = 0; w < NW - 1; ++w) {
                s0 += red[w][0][lane];
                s1 += red[w][1][lane];
            }
            const int c = (blockIdx.y * NC + j) * 16 + li;
            if (c < ncol) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = MfmaF64::orow(g, r);
                    if (i >= nr) continue;
                    const int row = T.rows[i];
                    double2 a = make_double2(s0[r], s1[r]);
                    if (F.leafbuf) {
                        if (s0_ptr) {
                            for (int q = s0_ptr[row]; q < s0_ptr[row + 1]; ++q)
                                a = cadd(a, far_value(F, s0_reps[q], c));
                        } else {
                            a = cadd(a, far_value(F, row, c));
                        }
                    }
                    y[int64_t(c) * nrows + row] = a;
                }
            }
        }
    }
}

// --------------------------------------------------------------------------
// Right-hand sides and far field
// --------------------------------------------------------------------------
struct QuadGeoArgs {
    const double* bez;
    const int* pg;
    const double* C1;
    const double* gl;
    int nel1, p, n;
    int64_t nelem;
};

// per element: sum_g w_g f(x_g) phi_a(x_g) for each direction, with
// f a = (rn d_n + rd) u_inc a = (rn i kappa d.n~ + rd a) u_inc
template <int P>
__global__ void rhs_elements(QuadGeoArgs A, const double* dirs, int ndir, double kappa, double2 rn, double2 rd,
                             double2* loc /* [ndir][E][NL] */) {
    constexpr int NL = (P + 1) * (P + 1);
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int dir = blockIdx.y;
    if (e >= A.nelem || dir >= ndir) return;
    const ElemRef R = elem_ref(A.bez, A.pg, A.nel1, e);
    const double* gx = A.gl + A.n * 2 * NGMAX;
    const double* gw = gx + NGMAX;
    const double* d = dirs + 3 * dir;
    double2 acc[NL];
    for (int a = 0; a < NL; ++a) acc[a] = make_double2(0, 0);
    for (int i = 0; i < A.n * A.n; ++i) {
        const double s = gx[i % A.n], t = gx[i / A.n];
        const double w = gw[i % A.n] * gw[i / A.n];
        GeoPt G;
        eval_geo(R.bez, R.pu, R.pv, s, t, G);
        double nt[3];
        cross3(G.fs, G.ft, nt);
        const double a = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
        const double dx = d[0] * G.x[0] + d[1] * G.x[1] + d[2] * G.x[2];
        const double dn = d[0] * nt[0] + d[1] * nt[1] + d[2] * nt[2];
        double sn, cs;
        sincos(kappa * dx, &sn, &cs);
        // c = rn i kappa d.n~ + rd a; f = c u_inc
        const double kd = kappa * dn;
        const double2 c = make_double2(-rn.y * kd + rd.x * a, rn.x * kd + rd.y * a);
        const double2 fval = make_double2(c.x * cs - c.y * sn, c.x * sn + c.y * cs);
        double bu[P + 1], bv[P + 1];
        eval_basis1<P>(A.C1 + R.ex * (P + 1) * (P + 1), s, bu, nullptr);
        eval_basis1<P>(A.C1 + R.ey * (P + 1) * (P + 1), t, bv, nullptr);
        for (int av = 0; av <= P; ++av)
            for (int au = 0; au <= P; ++au) {
                const double ph = w * bv[av] * bu[au];
                acc[av * (P + 1) + au].x = fma(ph, fval.x, acc[av * (P + 1) + au].x);
                acc[av * (P + 1) + au].y = fma(ph, fval.y, acc[av * (P + 1) + au].y);
            }
    }
    for (int a = 0; a < NL; ++a) loc[(int64_t(dir) * A.nelem + e) * NL + a] = acc[a];
}

// b[dir][row] = sum over representatives and their elements of loc (fixed order)
template <int P>
__global__ void rhs_gather(const double2* loc, int ndir, int64_t nelem, int nel1, int k, int64_t nrows,
                           const int* s0_ptr, const int* s0_reps, double2* b) {
    constexpr int NL = (P + 1) * (P + 1);
    const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int dir = blockIdx.y;
    if (row >= nrows) return;
    const int64_t kk = int64_t(k) * k;
    const int r0 = s0_ptr ? s0_ptr[row] : int(row);
    const int r1 = s0_ptr ? s0_ptr[row + 1] : int(row) + 1;
    double2 acc = make_double2(0, 0);
    for (int ri = r0; ri < r1; ++ri) {
        const int64_t i = s0_ptr ? s0_reps[ri] : ri;
        const int pj = int(i / kk), rem = int(i % kk), iv = rem / k, iu = rem % k;
        for (int ey = max(0, iv - P); ey <= min(iv, nel1 - 1); ++ey)
            for (int ex = max(0, iu - P); ex <= min(iu, nel1 - 1); ++ex) {
                const int64_t e = (int64_t(pj) * nel1 + ey) * nel1 + ex;
                acc = cadd(acc, loc[(int64_t(dir) * nelem + e) * NL + (iv - ey) * (P + 1) + (iu - ex)]);
            }
    }
    b[int64_t(dir) * nrows + row] = acc;
}

// boundary density and geometry at element quadrature points for far fields:
// geo[e][g] = (x(3), n~(3), a, w), dens[dir][e][g]
template <int P>
__global__ void density_points(QuadGeoArgs A, const double2* coef, int ndir, int64_t n,
                               const int* s2_to_s0, int k, double* geo, double2* dens) {
    constexpr int NL = (P + 1) * (P + 1);
    (void)NL;
    const int nqp = A.n * A.n;
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= A.nelem * nqp) return;
    const int64_t e = gid / nqp;
    const int i = int(gid % nqp);
    const ElemRef R = elem_ref(A.bez, A.pg, A.nel1, e);
    const double* gx = A.gl + A.n * 2 * NGMAX;
    const double* gw = gx + NGMAX;
    const double s = gx[i % A.n], t = gx[i / A.n];
    GeoPt G;
    eval_geo(R.bez, R.pu, R.pv, s, t, G);
    double nt[3];
    cross3(G.fs, G.ft, nt);
    double* o = geo + gid * 8;
    o[0] = G.x[0]; o[1] = G.x[1]; o[2] = G.x[2];
    o[3] = nt[0]; o[4] = nt[1]; o[5] = nt[2];
    o[6] = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
    o[7] = gw[i % A.n] * gw[i / A.n];
    double bu[P + 1], bv[P + 1];
    eval_basis1<P>(A.C1 + R.ex * (P + 1) * (P + 1), s, bu, nullptr);
    eval_basis1<P>(A.C1 + R.ey * (P + 1) * (P + 1), t, bv, nullptr);
    const int64_t patch = e / (int64_t(A.nel1) * A.nel1);
    for (int dir = 0; dir < ndir; ++dir) {
        double2 acc = make_double2(0, 0);
        for (int av = 0; av <= P; ++av)
            for (int au = 0; au <= P; ++au) {
                int64_t i2 = (patch * k + R.ey + av) * k + R.ex + au;
                int64_t c = s2_to_s0 ? s2_to_s0[i2] : i2;
                const double2 cv = coef[int64_t(dir) * n + c];
                const double ph = bv[av] * bu[au];
                acc.x = fma(ph, cv.x, acc.x);
                acc.y = fma(ph, cv.y, acc.y);
            }
        dens[(int64_t(dir) * A.nelem) * nqp + gid] = acc;
    }
}

__global__ __launch_bounds__(256) void farfield_sum(const double* geo, const double2* dens,
                                                    int64_t npts, const double* obs, int nobs,
                                                    double kappa, int hard, double2* uinf) {
    __shared__ double2 red[256];
    const int o = blockIdx.x, dir = blockIdx.y;
    const double* xh = obs + 3 * o;
    const double2* D = dens + int64_t(dir) * npts;
    double2 acc = make_double2(0, 0);
    for (int64_t i = threadIdx.x; i < npts; i += 256) {
        const double* g = geo + i * 8;
        const double ph = -kappa * (xh[0] * g[0] + xh[1] * g[1] + xh[2] * g[2]);
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double wt = g[7] * (hard ? (xh[0] * g[3] + xh[1] * g[4] + xh[2] * g[5]) : g[6]);
        const double2 z = cmul(make_double2(cs * wt, sn * wt), D[i]);
        acc = cadd(acc, z);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double c = 1.0 / (4.0 * M_PI);
        double2 r = red[0];
        // soft: -(1/4pi) S ; hard: -(i kappa / 4pi) S
        uinf[int64_t(dir) * nobs + o] = hard ? make_double2(c * kappa * r.y, -c * kappa * r.x)
                                             : make_double2(-c * r.x, -c * r.y);
    }
}

// kernel of the representation at one point pair, surface data g = (y, n~, a, w):
// soft -G a w, hard G (i kappa r - 1)/r^2 ((y - x).n~) w (used by both potential evaluations)
__device__ __forceinline__ double2 repr_kernel(const double* x, const double* g, double kappa, int hard) {
    const double d0 = g[0] - x[0], d1 = g[1] - x[1], d2 = g[2] - x[2];   // y - x
    const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double ir = 1.0 / r, kr = kappa * r;
    double sn, cs;
    sincos(kr, &sn, &cs);
    const double c4 = 0.07957747154594767 * ir;
    if (hard) {
        const double dn = (d0 * g[3] + d1 * g[4] + d2 * g[5]) * ir * ir * g[7];
        return make_double2(c4 * dn * (-cs - sn * kr), c4 * dn * (cs * kr - sn));
    }
    const double wa = -c4 * g[6] * g[7];
    return make_double2(wa * cs, wa * sn);
}

// scattered field at points off the boundary: soft u = -sum G a w dens,
// hard u = sum G (i kappa r - 1)/r^2 ((y - x).n~) w dens; one workgroup per
// (point, direction), fixed-order tree reduction
__global__ __launch_bounds__(256) void potential_sum(const double* geo, const double2* dens, int64_t npts,
                                                     const double* pts, int npt, double kappa, int hard,
                                                     double2* u) {
    __shared__ double2 red[256];
    const int o = blockIdx.x, dir = blockIdx.y;
    const double* x = pts + 3 * o;
    const double2* D = dens + int64_t(dir) * npts;
    double2 acc = make_double2(0, 0);
    for (int64_t i = threadIdx.x; i < npts; i += 256) acc = cfma(repr_kernel(x, geo + i * 8, kappa, hard), D[i], acc);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) u[int64_t(dir) * npt + o] = red[0];
}

// H^2 potential, sources: moments of the finest source clusters (s x s
// elements each) from the density at the quadrature points,
// mom[c][b (q+1) + a][r] = sum over the cluster's points of L_a(u) L_b(v) w rho
// / nel1^2, with (u, v) the point in the cluster's square and w / nel1^2 its
// weight in patch coordinates (the measure the interpolation nodes carry).
// Gauss rules of nqd >= 8 points per element and direction integrate these
// products (degree q + p in each direction) exactly, so these are the
// moments of the leaf-moment kernels.  One workgroup per (cluster, column).
constexpr int POTM_TILE = 256;
__global__ __launch_bounds__(256) void pot_leaf_moments(const double* __restrict__ geo,
                                                        const double2* __restrict__ dens, int64_t nqtot,
                                                        const double* __restrict__ gl, int nqd, int nel1, int lev,
                                                        int s, const double* __restrict__ tch, int q, int ncol,
                                                        double2* __restrict__ mom) {
    __shared__ double lu[POTM_TILE][QMAX + 1], lv[POTM_TILE][QMAX + 1];
    __shared__ double2 wd[POTM_TILE];
    const int64_t c = blockIdx.x;
    const int r = blockIdx.y, tid = threadIdx.x, q1 = q + 1, nq = q1 * q1;
    const int n = 1 << lev;
    const int64_t patch = c / (int64_t(n) * n);
    const int cy = int((c / n) % n), cx = int(c % n);
    const double* gx = gl + nqd * 2 * NGMAX;
    const int nqp = nqd * nqd, npt = s * s * nqp;
    const double inv = 1.0 / (double(nel1) * nel1);
    const double2* D = dens + int64_t(r) * nqtot;
    const int a = tid % q1, b = tid / q1;
    auto lag = [&](int j, double x) {
        double v = 1;
        for (int i = 0; i < q1; ++i)
            if (i != j) v *= (x - tch[i]) / (tch[j] - tch[i]);
        return v;
    };
    double2 acc = make_double2(0, 0);
    for (int t0 = 0; t0 < npt; t0 += POTM_TILE) {
        const int cnt = min(POTM_TILE, npt - t0);
        __syncthreads();   // the previous tile consumed
        for (int k = tid; k < cnt; k += blockDim.x) {
            const int li = t0 + k, el = li / nqp, gp = li % nqp, ex = el % s, ey = el / s;
            const int64_t gi = ((patch * nel1 + cy * s + ey) * nel1 + cx * s + ex) * nqp + gp;
            const double u = (ex + gx[gp % nqd]) / s, v = (ey + gx[gp / nqd]) / s;
            for (int j = 0; j < q1; ++j) {
                lu[k][j] = lag(j, u);
                lv[k][j] = lag(j, v);
            }
            const double w = geo[gi * 8 + 7] * inv;
            wd[k] = make_double2(w * D[gi].x, w * D[gi].y);
        }
        __syncthreads();
        if (tid < nq)
            for (int k = 0; k < cnt; ++k) {
                const double f = lu[k][a] * lv[k][b];
                acc.x = fma(f, wd[k].x, acc.x);
                acc.y = fma(f, wd[k].y, acc.y);
            }
    }
    if (tid < nq) mom[(c * nq + tid) * ncol + r] = acc;
}

// H^2 potential, far part: local expansion of every target box on its (q+1)^3
// Chebyshev nodes from the moments of its admissible source clusters, the
// kernel evaluated at node pairs (source nodes carry a and n~ like the
// coupling tiles).  One workgroup per (box, column); fixed summation order.
constexpr int POT_NODES_PER_THREAD = 6;   // (q+1)^3 <= 1331 for q <= 10
__global__ __launch_bounds__(256) void pot_box_m2l(const double* __restrict__ nodes, const double2* __restrict__ xh,
                                                   int q, const double* __restrict__ box_lo,
                                                   const double* __restrict__ box_hi, const double* __restrict__ tch,
                                                   const int* __restrict__ far_ptr, const int* __restrict__ far_src,
                                                   int ncol, double kappa, int hard, double2* __restrict__ lbox) {
    __shared__ double ys[(QMAX + 1) * (QMAX + 1)][8];
    __shared__ double2 xs[(QMAX + 1) * (QMAX + 1)];
    const int b = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
    const int q1 = q + 1, nq = q1 * q1, n3 = nq * q1;
    double X[POT_NODES_PER_THREAD][3];
    double2 acc[POT_NODES_PER_THREAD];
#pragma unroll
    for (int k = 0; k < POT_NODES_PER_THREAD; ++k) {
        acc[k] = make_double2(0, 0);
        const int a = tid + k * 256;
        const int ia[3] = {a % q1, (a / q1) % q1, a / nq};
        for (int c = 0; c < 3; ++c)
            X[k][c] = a < n3 ? box_lo[3 * b + c] + (box_hi[3 * b + c] - box_lo[3 * b + c]) * tch[ia[c]] : 0.0;
    }
    for (int f = far_ptr[b]; f < far_ptr[b + 1]; ++f) {
        const int64_t sc = far_src[f];
        __syncthreads();
        if (tid < nq) {
            const double* Y = nodes + (sc * nq + tid) * 16;
            ys[tid][0] = Y[0]; ys[tid][1] = Y[1]; ys[tid][2] = Y[2];
            ys[tid][3] = Y[3]; ys[tid][4] = Y[4]; ys[tid][5] = Y[5];
            ys[tid][6] = Y[6]; ys[tid][7] = 1.0;
            xs[tid] = xh[(sc * nq + tid) * ncol + r];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < POT_NODES_PER_THREAD; ++k) {
            if (tid + k * 256 >= n3) break;
            for (int j = 0; j < nq; ++j) acc[k] = cfma(repr_kernel(X[k], ys[j], kappa, hard), xs[j], acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < POT_NODES_PER_THREAD; ++k) {
        const int a = tid + k * 256;
        if (a < n3) lbox[(int64_t(b) * n3 + a) * ncol + r] = acc[k];
    }
}

// Interpolated box expansion lx (on the box's (q+1)^3 Chebyshev nodes) at point x
__device__ double2 pot_l2p(const double* x, const double* lo, const double* hi, const double* __restrict__ tch,
                           int q, const double2* lx) {
    const int q1 = q + 1;
    double w[3][QMAX + 1];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double t = (x[c] - lo[c]) / (hi[c] - lo[c]);
#pragma unroll
        for (int k = 0; k <= QMAX; ++k) {
            double v = 1;
#pragma unroll
            for (int j = 0; j <= QMAX; ++j)
                if (j != k && j < q1) v *= (t - tch[j]) / (tch[k < q1 ? k : 0] - tch[j]);
            w[c][k] = k < q1 ? v : 0.0;
        }
    }
    double2 acc = make_double2(0, 0);
    for (int az = 0; az < q1; ++az)
        for (int ay = 0; ay < q1; ++ay) {
            double2 row = make_double2(0, 0);
#pragma unroll
            for (int ax = 0; ax <= QMAX; ++ax)
                if (ax < q1) {
                    const double2 v = lx[(az * q1 + ay) * q1 + ax];
                    row.x = fma(w[0][ax], v.x, row.x);
                    row.y = fma(w[0][ax], v.y, row.y);
                }
            double wy = 0, wz = 0;
#pragma unroll
            for (int k = 0; k <= QMAX; ++k) {
                if (k == ay) wy = w[1][k];
                if (k == az) wz = w[2][k];
            }
            const double wyz = wy * wz;
            acc.x = fma(wyz, row.x, acc.x);
            acc.y = fma(wyz, row.y, acc.y);
        }
    return acc;
}

// H^2 potential, per point: the box expansion interpolated at the point (tensor
// Lagrange on the box's Chebyshev nodes), plus the interpolation nodes of the
// clusters that act on the points directly (each node a source point carrying
// the cluster's moment), plus direct quadrature over the elements of the box's
// inadmissible finest clusters (level L, s x s elements each).  Source points
// are staged in LDS a tile at a time and shared by the box's points.  One workgroup per (box, column); a box of
// few points gives each point a group of lanes (a power of two) that split
// every tile and add their partial sums in a fixed order, so a column's result
// does not depend on the others.
constexpr int POT_TILE = 256;   // source points per LDS tile
__global__ __launch_bounds__(POT_LEAF_POINTS) void pot_l2p_near(
    const double* __restrict__ pts, const int* __restrict__ perm, const int* __restrict__ box_ptr,
    const double* __restrict__ box_lo, const double* __restrict__ box_hi, const double* __restrict__ tch, int q,
    const double2* __restrict__ lbox, int ncol, const int* __restrict__ m2p_ptr, const int* __restrict__ m2p_src,
    const double* __restrict__ nodes, const double2* __restrict__ xh, const int* __restrict__ near_ptr,
    const int* __restrict__ near_leaf, int d, int L, int nel1, int nqp, const double* __restrict__ geo,
    const double2* __restrict__ dens, int64_t nqtot, double kappa, int hard, int npt, double2* __restrict__ u) {
    // the box expansion, the source tiles and the partial sums share the LDS (one after the other)
    constexpr int LX = (QMAX + 1) * (QMAX + 1) * (QMAX + 1), TL = POT_TILE * 5;
    static_assert(TL >= POT_LEAF_POINTS, "partial sums fit the tile space");
    __shared__ double2 smem[LX > TL ? LX : TL];
    double2* lx = smem;
    double(*tg)[8] = reinterpret_cast<double(*)[8]>(smem);     // [POT_TILE][8]
    double2* td = smem + POT_TILE * 4;                           // [POT_TILE]
    const int b = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
    const int q1 = q + 1, nq = q1 * q1, n3 = nq * q1;
    const bool has_far = lbox != nullptr;
    const double2* D = dens + int64_t(r) * nqtot;
    const int n = 1 << L, s = 1 << d, per_leaf = s * s * nqp;
    const int p0 = box_ptr[b], p1 = box_ptr[b + 1];
    // lanes per point: the largest power of two gs with gs * points <= the workgroup
    int gs = 1;
    while (gs < POT_LEAF_POINTS && 2 * gs * (p1 - p0) <= POT_LEAF_POINTS) gs *= 2;
    const int slot = tid / gs, lane = tid % gs, per_round = POT_LEAF_POINTS / gs;
    const int f0 = m2p_ptr[b], nm2p = (m2p_ptr[b + 1] - f0) * nq;
    // (a box at the depth cap may hold more points than threads)
    for (int base = p0; base < p1; base += per_round) {
        const int i = base + slot;
        const bool mine = i < p1;
        const int pi = mine ? perm[i] : 0;
        const double x[3] = {pts[3 * pi], pts[3 * pi + 1], pts[3 * pi + 2]};
        double2 acc = make_double2(0, 0);
        __syncthreads();   // the previous round's tiles and partial sums consumed
        if (has_far) {
            for (int a = tid; a < n3; a += POT_LEAF_POINTS) lx[a] = lbox[(int64_t(b) * n3 + a) * ncol + r];
            __syncthreads();
            if (mine && lane == 0) acc = pot_l2p(x, box_lo + 3 * b, box_hi + 3 * b, tch, q, lx);
            __syncthreads();   // lx consumed before the tiles overwrite it
        }
        // cluster nodes evaluated at the points: position, n~, a, weight 1, the moment as density
        for (int t0 = 0; t0 < nm2p; t0 += POT_TILE) {
            const int cnt = min(POT_TILE, nm2p - t0);
            for (int k = tid; k < cnt; k += POT_LEAF_POINTS) {
                const int64_t sc = m2p_src[f0 + (t0 + k) / nq];
                const int64_t ni = sc * nq + (t0 + k) % nq;
#pragma unroll
                for (int c = 0; c < 7; ++c) tg[k][c] = nodes[ni * 16 + c];
                tg[k][7] = 1.0;
                td[k] = xh[ni * ncol + r];
            }
            __syncthreads();
            if (mine)
                for (int k = lane; k < cnt; k += gs) acc = cfma(repr_kernel(x, tg[k], kappa, hard), td[k], acc);
            __syncthreads();
        }
        for (int f = near_ptr[b]; f < near_ptr[b + 1]; ++f) {
            const int64_t loc = near_leaf[f];
            const int64_t patch = loc / (int64_t(n) * n);
            const int cy = int((loc / n) % n), cx = int(loc % n);
            for (int t0 = 0; t0 < per_leaf; t0 += POT_TILE) {
                const int cnt = min(POT_TILE, per_leaf - t0);
                for (int k = tid; k < cnt; k += POT_LEAF_POINTS) {
                    const int li = t0 + k, el = li / nqp, g = li % nqp;
                    const int64_t e = (patch * nel1 + cy * s + el / s) * nel1 + cx * s + el % s;
                    const int64_t gi = e * nqp + g;
#pragma unroll
                    for (int c = 0; c < 8; ++c) tg[k][c] = geo[gi * 8 + c];
                    td[k] = D[gi];
                }
                __syncthreads();
                if (mine)
                    for (int k = lane; k < cnt; k += gs) acc = cfma(repr_kernel(x, tg[k], kappa, hard), td[k], acc);
                __syncthreads();
            }
        }
        if (gs == 1) {
            if (mine) u[int64_t(r) * npt + pi] = acc;
        } else {
            smem[tid] = acc;
            __syncthreads();
            if (mine && lane == 0) {
                for (int l = 1; l < gs; ++l) acc = cadd(acc, smem[tid + l]);
                u[int64_t(r) * npt + pi] = acc;
            }
        }
    }
}

// ==========================================================================
// host launchers
// ==========================================================================
namespace {

// device buffers, charged to the calling entry point's context (dev_malloc);
// acct (if given) also counts them for the handle that owns them
template <class T>
igb_status upload(DevBuf& b, const T* src, size_t n, size_t* acct) {
    if (igb_status st = dev_malloc(b, n * sizeof(T), "device upload")) return st;
    if (n == 0) return IGB_OK;
    if (acct) *acct += b.bytes;
    if (src) IGB_HIP(hipMemcpy(b.ptr, src, n * sizeof(T), hipMemcpyHostToDevice));
    return IGB_OK;
}

igb_status alloc(DevBuf& b, size_t bytes, size_t* acct) {
    if (igb_status st = dev_malloc(b, bytes, "device allocation")) return st;
    if (acct) *acct += b.bytes;
    return IGB_OK;
}

std::vector<double> gauss_table() {
    // Gauss-Legendre nodes / weights on [0,1] for orders 1..NGMAX by Newton's
    // iteration on the Legendre recurrence
    std::vector<double> t((NGMAX + 1) * 2 * NGMAX, 0.0);
    for (int n = 1; n <= NGMAX; ++n) {
        for (int i = 0; i < n; ++i) {
            double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
            double dp = 1;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1, p1 = x;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                if (n == 1) { p1 = x; p0 = 1; }
                dp = n * (x * p1 - p0) / (x * x - 1);
                double dx = p1 / dp;
                x -= dx;
                if (std::fabs(dx) < 1e-16) break;
            }
            double p0 = 1, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1);
            t[n * 2 * NGMAX + i] = 0.5 * (1 - x);
            t[n * 2 * NGMAX + NGMAX + i] = 1.0 / ((1 - x * x) * dp * dp);
        }
    }
    return t;
}

void gauss01_host(int n, std::vector<double>& x, std::vector<double>& w) {
    static std::vector<double> tab = gauss_table();
    n = std::max(1, std::min(n, NGMAX));
    x.assign(tab.begin() + n * 2 * NGMAX, tab.begin() + n * 2 * NGMAX + n);
    w.assign(tab.begin() + n * 2 * NGMAX + NGMAX, tab.begin() + n * 2 * NGMAX + NGMAX + n);
}

// Duffy-type rules on [0,1]^4 as (s1, s2, r1, r2, w) for the three touching
// configurations (identical element; shared edge s2 = r2 = 0 with s1 = r1;
// shared vertex at the origin).  Each coordinate pair (s, r) of the identical
// and edge cases is written as offset u = |r - s| and position w in [0,1]
// (Jacobian 1 - u); the singular corner of the remaining cube is removed by
// splitting it into simplices / pyramids along its largest coordinate rho.
std::vector<double> duffy_rule(int cls, int n) {
    std::vector<double> gx, gw;
    gauss01_host(n, gx, gw);
    std::vector<double> out;
    auto split = [](double u, double w, int sig, double& s, double& r) {
        double base = w * (1 - u);
        if (sig > 0) { s = base; r = base + u; }
        else { s = base + u; r = base; }
    };
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            for (int c = 0; c < n; ++c)
                for (int d = 0; d < n; ++d) {
                    const double rho = gx[a], t1 = gx[b], t2 = gx[c], t3 = gx[d];
                    const double W = gw[a] * gw[b] * gw[c] * gw[d];
                    if (cls == 2) {  // identical: 2 x 2 signs x 2 triangles
                        for (int sg = 0; sg < 4; ++sg)
                            for (int tri = 0; tri < 2; ++tri) {
                                double u1 = tri ? rho * t1 : rho, u2 = tri ? rho : rho * t1;
                                double s1, r1, s2, r2;
                                split(u1, t2, (sg & 1) ? -1 : 1, s1, r1);
                                split(u2, t3, (sg & 2) ? -1 : 1, s2, r2);
                                out.insert(out.end(), {s1, s2, r1, r2, W * (1 - u1) * (1 - u2) * rho});
                            }
                    } else if (cls == 1) {  // edge: 2 signs x 3 pyramids
                        for (int sg = 0; sg < 2; ++sg)
                            for (int pyr = 0; pyr < 3; ++pyr) {
                                double u1, s2, r2;
                                if (pyr == 0) { u1 = rho; s2 = rho * t1; r2 = rho * t2; }
                                else if (pyr == 1) { u1 = rho * t1; s2 = rho; r2 = rho * t2; }
                                else { u1 = rho * t1; s2 = rho * t2; r2 = rho; }
                                double s1, r1;
                                split(u1, t3, sg ? -1 : 1, s1, r1);
                                out.insert(out.end(), {s1, s2, r1, r2, W * (1 - u1) * rho * rho});
                            }
                    } else {  // vertex: 4 pyramids
                        for (int pyr = 0; pyr < 4; ++pyr) {
                            double c4[4];
                            double rest[3] = {rho * t1, rho * t2, rho * t3};
                            for (int i = 0, j = 0; i < 4; ++i) c4[i] = (i == pyr) ? rho : rest[j++];
                            out.insert(out.end(), {c4[0], c4[1], c4[2], c4[3], W * rho * rho * rho});
                        }
                    }
                }
    return out;
}

}  // namespace

igb_status upload_geometry(igb_geom g) {
    size_t acct = 0;
    igb_status st;
    if ((st = upload(g->d_bez, g->bez.data(), g->bez.size(), &acct))) return st;
    if ((st = upload(g->d_pg, g->pg.data(), g->pg.size(), &acct))) return st;
    if ((st = upload(g->d_C1, g->C1.data(), g->C1.size(), &acct))) return st;
    g->dev_bytes = acct;
    return IGB_OK;
}

// f(std::integral_constant<int, P>) for the degree p = 0..PMAX of the discrete spaces
template <class F>
static igb_status with_degree(int p, const char* who, F&& f) {
    switch (p) {
        case 0: return f(std::integral_constant<int, 0>{});
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
        default:
            set_error("%s: spline degree p = %d not built (0 <= p <= %d)", who, p, PMAX);
            return IGB_ERR_UNSUPPORTED;
    }
}

// orders of the GPU rules (see near_classify for the regular ones)
constexpr int NSING_IDENT = 7, NSING_EDGE = 8, NSING_VERTEX = 9, MASS_ORDER = 6;

template <int P, bool HARD>
static igb_status near_launch(igb_op op, hipStream_t s) {
    igb_geom g = op->geom;
    constexpr int NL = (P + 1) * (P + 1);
    const int64_t E = g->nelem;
    const int64_t npairs = op->near_ptr[E];
    size_t* acct = &op->dev_bytes;
    igb_status st;
    // pair arrays
    std::vector<int> pe(npairs);
    for (int64_t e = 0; e < E; ++e)
        for (int64_t k = op->near_ptr[e]; k < op->near_ptr[e + 1]; ++k) pe[k] = int(e);
    DevBuf d_pe, d_pf, d_kind, d_gl, d_rules[3], d_list, d_stage;
    if ((st = upload(d_pe, pe.data(), pe.size(), nullptr))) return st;
    if ((st = upload(d_pf, op->near_src.data(), op->near_src.size(), nullptr))) return st;
    if ((st = upload(d_kind, op->near_kind.data(), op->near_kind.size(), nullptr))) return st;
    std::vector<double> gl = gauss_table();
    if ((st = upload(d_gl, gl.data(), gl.size(), nullptr))) return st;
    const int raise = op->prm.quad_extra + kd_boost(op->kd_elem) + aspect_boost(op->aspect_max);
    const int ord[3] = {std::min(NGMAX, NSING_VERTEX + raise), std::min(NGMAX, NSING_EDGE + raise),
                        std::min(NGMAX, NSING_IDENT + raise)};
    NearArgs A{};
    for (int c = 0; c < 3; ++c) {
        std::vector<double> r = duffy_rule(c, ord[c]);
        if ((st = upload(d_rules[c], r.data(), r.size(), nullptr))) return st;
        A.rule[c] = d_rules[c].as<double>();
        A.rule_n[c] = int(r.size() / 5);
    }
    if ((st = upload(op->d_near_ptr, op->near_ptr.data(), op->near_ptr.size(), acct))) return st;
    if ((st = upload(op->d_near_src, op->near_src.data(), op->near_src.size(), acct))) return st;
    if ((st = upload(op->d_rowptr, op->row_ptr.data(), op->row_ptr.size(), acct))) return st;
    if ((st = upload(op->d_col, op->col.data(), op->col.size(), acct))) return st;
    if ((st = upload(op->d_dcol, op->near_dcol.data(), op->near_dcol.size(), acct))) return st;
    if ((st = upload(op->d_row_coff, op->row_coff.data(), op->row_coff.size(), acct))) return st;
    if ((st = upload(op->d_near_wgs, op->near_wgs.data(), op->near_wgs.size(), acct))) return st;
    if ((st = upload(op->d_near_grp_rows, op->near_grp_rows.data(), op->near_grp_rows.size(), acct))) return st;
    if ((st = alloc(op->d_val, op->nnz * sizeof(double2), acct))) return st;
    IGB_HIP(hipMemsetAsync(op->d_val.ptr, 0, op->nnz * sizeof(double2), s));

    A.bez = g->d_bez.as<double>();
    A.pg = g->d_pg.as<int>();
    A.C1 = g->d_C1.as<double>();
    A.gl = d_gl.as<double>();
    A.pair_e = d_pe.as<int>();
    A.pair_f = d_pf.as<int>();
    A.pair_kind = d_kind.as<int>();
    A.nel1 = g->nel1;
    A.kappa = op->kappa;
    A.eta = op->eta;
    A.mix = op->mix;
    A.hmix = op->hmix;
    A.cm = op->cm;
    A.mass_order = MASS_ORDER;

    // chunks of target elements with a bounded staging buffer
    const int64_t max_slots = std::max<int64_t>(int64_t(1) << 22, 1);  // 4M pairs
    if ((st = alloc(d_stage, size_t(std::min(npairs, max_slots)) * NL * NL * sizeof(double2), nullptr)))
        return st;
    if ((st = alloc(d_list, size_t(std::min(npairs, max_slots)) * sizeof(int), nullptr))) return st;
    A.stage = d_stage.as<double2>();
    const bool hard = op->bc == IGB_HARD;
    int64_t e0 = 0;
    std::vector<int> reg, reg_big, sing;
    auto points = [](int kind) {
        return std::max(((kind >> 8) & 15) * ((kind >> 12) & 15), ((kind >> 16) & 15) * ((kind >> 20) & 15));
    };
    while (e0 < E) {
        int64_t e1 = e0;
        while (e1 < E && op->near_ptr[e1 + 1] - op->near_ptr[e0] <= max_slots) ++e1;
        if (e1 == e0) {
            set_error("assemble_nearfield: one element has more near pairs than the staging buffer");
            return IGB_ERR_UNSUPPORTED;
        }
        const int64_t k0 = op->near_ptr[e0], k1 = op->near_ptr[e1];
        reg.clear();
        reg_big.clear();
        sing.clear();
        for (int64_t k = k0; k < k1; ++k) {
            const int kind = op->near_kind[k];
            ((kind & 15) != 0 ? sing : points(kind) <= 49 ? reg : reg_big).push_back(int(k));
        }
        A.slot0 = k0;
        // regular pairs with at most 49 points per element, then the larger regular
        // rules, then the touching pairs
        std::vector<int> lst(reg);
        lst.insert(lst.end(), reg_big.begin(), reg_big.end());
        lst.insert(lst.end(), sing.begin(), sing.end());
        if (!lst.empty())
            IGB_HIP(hipMemcpyAsync(d_list.ptr, lst.data(), lst.size() * sizeof(int), hipMemcpyHostToDevice, s));
        if (!reg.empty()) {
            A.list = d_list.as<int>();
            A.nlist = int64_t(reg.size());
            hipLaunchKernelGGL((near_regular<P, HARD, 49>), dim3(unsigned(reg.size())), dim3(NEAR_THREADS), 0, s, A);
            IGB_HIP(hipGetLastError());
        }
        if (!reg_big.empty()) {
            A.list = d_list.as<int>() + reg.size();
            A.nlist = int64_t(reg_big.size());
            hipLaunchKernelGGL((near_regular<P, HARD, REG_POINTS_MAX>), dim3(unsigned(reg_big.size())),
                               dim3(NEAR_THREADS), 0, s, A);
            IGB_HIP(hipGetLastError());
        }
        if (!sing.empty()) {
            A.list = d_list.as<int>() + reg.size() + reg_big.size();
            A.nlist = int64_t(sing.size());
            hipLaunchKernelGGL((near_singular<P, HARD>), dim3(unsigned(sing.size())), dim3(NEAR_THREADS), 0, s, A);
            IGB_HIP(hipGetLastError());
        }
        // rows touched by the chunk's target elements
        int64_t rlo = op->N, rhi = -1;
        for (int64_t e = e0; e < e1; ++e) {
            const int nel1 = g->nel1, k = g->k;
            int j = int(e / (int64_t(nel1) * nel1));
            int rem = int(e % (int64_t(nel1) * nel1));
            int ey = rem / nel1, ex = rem % nel1;
            for (int av = 0; av <= P; ++av)
                for (int au = 0; au <= P; ++au) {
                    int64_t i2 = (int64_t(j) * k + ey + av) * k + ex + au;
                    int64_t r = hard ? g->s2_to_s0[i2] : i2;
                    rlo = std::min(rlo, r);
                    rhi = std::max(rhi, r);
                }
        }
        CsrArgs C{};
        C.row_ptr = op->d_rowptr.as<int64_t>();
        C.col = op->d_col.as<int>();
        C.val = op->d_val.as<double2>();
        C.near_ptr = op->d_near_ptr.as<int64_t>();
        C.near_src = op->d_near_src.as<int>();
        C.stage = d_stage.as<double2>();
        C.slot0 = k0;
        C.e_lo = e0;
        C.e_hi = e1;
        C.s0_ptr = hard ? op->d_s0_ptr.as<int>() : nullptr;
        C.s0_reps = hard ? op->d_s0_reps.as<int>() : nullptr;
        C.row0 = rlo;
        C.nel1 = g->nel1;
        C.k = g->k;
        if (rhi >= rlo) {
            hipLaunchKernelGGL(near_gather_csr<P>, dim3(unsigned(rhi - rlo + 1)), dim3(256), 0, s, C);
            IGB_HIP(hipGetLastError());
        }
        IGB_HIP(hipStreamSynchronize(s));
        e0 = e1;
    }
    return IGB_OK;
}

igb_status assemble_near_device(igb_op op, hipStream_t s) {
    igb_geom g = op->geom;
    size_t* acct = &op->dev_bytes;
    igb_status st;
    if ((st = upload(op->d_s2_to_s0, g->s2_to_s0.data(), g->s2_to_s0.size(), acct))) return st;
    if (g->n0 > 0) {
        if ((st = upload(op->d_s0_ptr, g->s0_ptr.data(), g->s0_ptr.size(), acct))) return st;
        if ((st = upload(op->d_s0_reps, g->s0_reps.data(), g->s0_reps.size(), acct))) return st;
    }
    auto t0 = std::chrono::steady_clock::now();
    const bool hard = op->bc == IGB_HARD;
    st = with_degree(g->p, "assemble_nearfield", [&](auto deg) {
        constexpr int P = decltype(deg)::value;
        if constexpr (P == 0)
            return near_launch<0, false>(op, s);  // S^0 needs p >= 1: checked at the entry point
        else
            return hard ? near_launch<P, true>(op, s) : near_launch<P, false>(op, s);
    });
    if (!st && (op->prm.precision == IGB_FP64 || op->prm.precision == IGB_MIX_FP32) && op->nnz > 0 &&
        !op->near_tiles.empty()) {
        // fp64 copy of the near field in the tile layout: fp64 operators' blocks of
        // >= 16 columns, fp32 operators' reduced-precision products (every block size)
        const int64_t nt = int64_t(op->near_tiles.size());
        if ((st = upload(op->d_near_tiles, op->near_tiles.data(), op->near_tiles.size(), acct))) return st;
        if ((st = upload(op->d_near_tile_cols, op->near_tile_cols.data(), op->near_tile_cols.size(), acct))) return st;
        if ((st = alloc(op->d_val64, size_t(op->near_tile_vals) * sizeof(double2), acct))) return st;
        hipLaunchKernelGGL(near_tile_values64, dim3(unsigned(nt)), dim3(64), 0, s, op->d_near_tiles.as<NearTile>(),
                           op->d_near_tile_cols.as<int>(), op->d_rowptr.as<int64_t>(), op->d_col.as<int>(),
                           op->d_val.as<double2>(), op->d_val64.as<double2>());
        IGB_HIP(hipGetLastError());
        IGB_HIP(hipStreamSynchronize(s));
    }
    if (!st && op->prm.precision == IGB_MIX_BF16 && op->nnz > 0) {
        // fp32 copy of the near field for the inner matvecs of the bf16 refinement (whose
        // inner solves stop at 1e-3; the fp32 operator's inner solves aim at the full
        // tolerance, below what fp32 columns allow, and keep the fp64 near product),
        // in the tile layout of the matrix-core near product
        const int64_t nt = int64_t(op->near_tiles.size());
        if ((st = upload(op->d_near_tiles, op->near_tiles.data(), op->near_tiles.size(), acct))) return st;
        if ((st = upload(op->d_near_tile_cols, op->near_tile_cols.data(), op->near_tile_cols.size(), acct))) return st;
        if ((st = alloc(op->d_val_lo, size_t(op->near_tile_vals) * sizeof(float2), acct))) return st;
        hipLaunchKernelGGL(near_tile_values, dim3(unsigned(nt)), dim3(64), 0, s, op->d_near_tiles.as<NearTile>(),
                           op->d_near_tile_cols.as<int>(), op->d_rowptr.as<int64_t>(), op->d_col.as<int>(),
                           op->d_val.as<double2>(), op->d_val_lo.as<float2>());
        IGB_HIP(hipGetLastError());
        IGB_HIP(hipStreamSynchronize(s));
    }
    auto t1 = std::chrono::steady_clock::now();
    op->t_assembly_near = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return st;
}

igb_status assemble_far_device(igb_op op, hipStream_t s) {
    igb_geom g = op->geom;
    size_t* acct = &op->dev_bytes;
    igb_status st;
    const int q = op->q, q1 = q + 1, nq = op->nq, L = op->L, d = op->d, p = g->p;
    auto t0 = std::chrono::steady_clock::now();
    // Chebyshev nodes, transfers T1[bit][g][a] = L_a((bit + t_g)/2), 1-D leaf moments
    std::vector<double> t(q1);
    cheb_nodes(q, t.data());
    auto lag = [&](int a, double x) {
        double v = 1;
        for (int b = 0; b < q1; ++b)
            if (b != a) v *= (x - t[b]) / (t[a] - t[b]);
        return v;
    };
    std::vector<double> T1(2 * q1 * q1);
    for (int bit = 0; bit < 2; ++bit)
        for (int gg = 0; gg < q1; ++gg)
            for (int a = 0; a < q1; ++a) T1[(bit * q1 + gg) * q1 + a] = lag(a, 0.5 * (bit + t[gg]));
    // m1[kind][cx][a][i] = int_{leaf cx} L_a(x) b^{(kind)}_{cx*s + i}(x) dx over the
    // window of the leaf's B-splines, kind 0 values / 1 derivatives
    const int s1 = 1 << d, w = s1 + p, nleaf1 = 1 << L, nel1 = g->nel1;
    const int64_t stride_kind = int64_t(nleaf1) * q1 * w;
    std::vector<double> m1(2 * stride_kind, 0.0);
    {
        std::vector<double> gx, gw;
        const int ng = std::min(NGMAX, (q + p) / 2 + 2);
        gauss01_host(ng, gx, gw);
        for (int cx = 0; cx < nleaf1; ++cx)
            for (int el = 0; el < s1; ++el) {
                const int ex = cx * s1 + el;
                const double* C = &g->C1[size_t(ex) * (p + 1) * (p + 1)];
                for (int gi = 0; gi < ng; ++gi) {
                    const double sl = gx[gi];
                    const double xr = (el + sl) / s1;  // position in the leaf's [0,1]
                    double b[4], db[4];
                    // Bernstein on the element, then extraction to B-splines
                    {
                        const double tt = 1 - sl;
                        if (p == 1) { b[0] = tt; b[1] = sl; db[0] = -1; db[1] = 1; }
                        else if (p == 2) { b[0] = tt * tt; b[1] = 2 * sl * tt; b[2] = sl * sl; db[0] = -2 * tt; db[1] = 2 * (tt - sl); db[2] = 2 * sl; }
                        else if (p == 3) { b[0] = tt * tt * tt; b[1] = 3 * sl * tt * tt; b[2] = 3 * sl * sl * tt; b[3] = sl * sl * sl; db[0] = -3 * tt * tt; db[1] = 3 * tt * tt - 6 * sl * tt; db[2] = 6 * sl * tt - 3 * sl * sl; db[3] = 3 * sl * sl; }
                        else { b[0] = 1; db[0] = 0; }
                    }
                    for (int a = 0; a <= p; ++a) {
                        double v = 0, dv = 0;
                        for (int kk = 0; kk <= p; ++kk) {
                            v += C[a * (p + 1) + kk] * b[kk];
                            dv += C[a * (p + 1) + kk] * db[kk];
                        }
                        dv *= nel1;  // d/du = 2^m d/ds
                        const int iloc = el + a;  // window index of b_{ex+a}
                        for (int aa = 0; aa < q1; ++aa) {
                            const double la = lag(aa, xr) * gw[gi] / nel1;
                            m1[(int64_t(cx) * q1 + aa) * w + iloc] += la * v;
                            m1[stride_kind + (int64_t(cx) * q1 + aa) * w + iloc] += la * dv;
                        }
                    }
                }
            }
    }
    if ((st = upload(op->d_T, T1.data(), T1.size(), acct))) return st;
    {
        // composite downward transfers: delta = 1..L levels down at offset pos,
        // Tc[2^delta - 2 + pos][g][a] = L_a((pos + t_g) / 2^delta)
        std::vector<double> Tc(size_t((int64_t(2) << L) - 2) * q1 * q1 + 1);
        for (int dl = 1; dl <= L; ++dl)
            for (int pos = 0; pos < (1 << dl); ++pos)
                for (int gg = 0; gg < q1; ++gg)
                    for (int a = 0; a < q1; ++a)
                        Tc[((int64_t((1 << dl) - 2 + pos) * q1 + gg) * q1 + a)] =
                            lag(a, (pos + t[gg]) / double(1 << dl));
        if ((st = upload(op->d_Tc, Tc.data(), Tc.size(), acct))) return st;
    }
    if ((st = upload(op->d_m1, m1.data(), m1.size(), acct))) return st;
    DevBuf d_t, d_cluoff;
    if ((st = upload(d_t, t.data(), t.size(), nullptr))) return st;
    if ((st = upload(d_cluoff, op->clu_off.data(), op->clu_off.size(), nullptr))) return st;
    if ((st = alloc(op->d_nodes, size_t(op->nclusters) * nq * 16 * sizeof(double), acct))) return st;
    {
        const int64_t tot = op->nclusters * nq;
        hipLaunchKernelGGL(node_geometry, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s,
                           g->d_bez.as<double>(), g->d_pg.as<int>(), g->nel1, g->npatch, L,
                           d_cluoff.as<int64_t>(), d_t.as<double>(), q, op->d_nodes.as<double>());
        IGB_HIP(hipGetLastError());
    }
    // far pair lists (global cluster indices)
    std::vector<int> ptg(op->nfar), psg(op->nfar);
    for (int l = 0; l <= L; ++l) {
        const FarLevel& F = op->far[l];
        const int64_t nc = clusters_on_level(g->npatch, l);
        for (int64_t tt = 0; tt < nc; ++tt)
            for (int i = F.tgt_ptr[tt]; i < F.tgt_ptr[tt + 1]; ++i) {
                ptg[F.pair_off + i] = int(op->clu_off[l] + tt);
                psg[F.pair_off + i] = int(op->clu_off[l] + F.src[i]);
            }
    }
    DevBuf d_ptg;
    if ((st = upload(d_ptg, ptg.data(), ptg.size(), nullptr))) return st;
    if ((st = upload(op->d_far_src, psg.data(), psg.size(), acct))) return st;
    const bool hard = op->bc == IGB_HARD;
    const bool otf = op->prm.far_on_the_fly != 0;
    const size_t fp64_tile_bytes = size_t(op->nfar) * nq * nq * sizeof(double2) * (hard ? 2 : 1);
    if (!otf) {
        // slack after the last tile for the matrix-core k-block overrun (fp64 operators)
        if ((st = alloc(op->d_coupling, fp64_tile_bytes + lo_slack(op), acct))) return st;
        IGB_HIP(hipMemsetAsync(static_cast<char*>(op->d_coupling.ptr) + fp64_tile_bytes, 0, lo_slack(op), s));
    }
    if (op->nfar > 0 && !otf) {
        if (hard)
            hipLaunchKernelGGL(coupling_hard, dim3(unsigned(std::min<int64_t>(op->nfar, 1 << 20))), dim3(256), 0, s,
                               op->d_nodes.as<double>(),
                               d_ptg.as<int>(), op->d_far_src.as<int>(), op->nfar, nq, op->kappa,
                               op->d_coupling.as<double2>());
        else
            hipLaunchKernelGGL(coupling_soft, dim3(unsigned(std::min<int64_t>(op->nfar, 1 << 20))), dim3(256), 0, s,
                               op->d_nodes.as<double>(),
                               d_ptg.as<int>(), op->d_far_src.as<int>(), op->nfar, nq, op->kappa, op->mix,
                               op->d_coupling.as<double2>());
        IGB_HIP(hipGetLastError());
    }
    if (op->nfar > 0 && !otf && !hard && op->prm.far_recompress_tol > 0) {
        // factors of every tile: count the terms, lay them out, then write them
        if ((st = alloc(op->d_lr_rank, size_t(op->nfar) * sizeof(int), acct))) return st;
        const dim3 grid(unsigned(std::min<int64_t>(op->nfar, 1 << 16)));
        hipLaunchKernelGGL(tile_rrqr, grid, dim3(256), 0, s, op->d_coupling.as<double2>(), op->nfar, nq,
                           op->prm.far_recompress_tol, op->d_lr_rank.as<int>(), nullptr, nullptr);
        IGB_HIP(hipGetLastError());
        std::vector<int> rk(op->nfar);
        IGB_HIP(hipMemcpyAsync(rk.data(), op->d_lr_rank.ptr, rk.size() * sizeof(int), hipMemcpyDeviceToHost, s));
        IGB_HIP(hipStreamSynchronize(s));
        std::vector<int64_t> off(op->nfar);
        int64_t tot = 0;
        for (int64_t i = 0; i < op->nfar; ++i) {
            off[i] = tot;
            tot += int64_t(2) * rk[i] * nq;
        }
        op->lr_entries = tot;
        if ((st = upload(op->d_lr_off, off.data(), off.size(), acct))) return st;
        // at least 64 entries: the product kernel's idle pairs read the first nq
        if ((st = alloc(op->d_lr, size_t(std::max<int64_t>(tot, 64)) * sizeof(double2), acct))) return st;
        hipLaunchKernelGGL(tile_rrqr, grid, dim3(256), 0, s, op->d_coupling.as<double2>(), op->nfar, nq,
                           op->prm.far_recompress_tol, op->d_lr_rank.as<int>(), op->d_lr_off.as<int64_t>(),
                           op->d_lr.as<double2>());
        IGB_HIP(hipGetLastError());
    }
    if (op->nfar > 0 && op->prm.precision != IGB_FP64) {
        const int ntile = hard ? 2 : 1;
        const bool f32 = op->prm.precision == IGB_MIX_FP32;
        const int nkc = lo_nkc(op);
        const int64_t ne = op->nfar * ntile * nkc * nq * lo_epl(op);
        const size_t esz = lo_esz(op), slack = lo_slack(op);
        if ((st = alloc(op->d_coupling_lo, size_t(ne) * esz + slack, acct))) return st;
        IGB_HIP(hipMemsetAsync(static_cast<char*>(op->d_coupling_lo.ptr) + size_t(ne) * esz, 0, slack, s));
        const dim3 grid(unsigned(std::min<int64_t>((ne + 255) / 256, int64_t(1) << 20))), blk(256);
        const double* nd = op->d_nodes.as<double>();
        const int* pt = d_ptg.as<int>();
        const int* ps = op->d_far_src.as<int>();
        if (f32 && hard)
            hipLaunchKernelGGL((coupling_lo<float2, true>), grid, blk, 0, s, nd, pt, ps, op->nfar, nq, nkc, op->kappa,
                               op->mix, op->d_coupling_lo.as<float2>());
        else if (f32)
            hipLaunchKernelGGL((coupling_lo<float2, false>), grid, blk, 0, s, nd, pt, ps, op->nfar, nq, nkc, op->kappa,
                               op->mix, op->d_coupling_lo.as<float2>());
        else if (hard)
            hipLaunchKernelGGL((coupling_lo<bf16x2, true>), grid, blk, 0, s, nd, pt, ps, op->nfar, nq, nkc, op->kappa,
                               op->mix, op->d_coupling_lo.as<bf16x2>());
        else
            hipLaunchKernelGGL((coupling_lo<bf16x2, false>), grid, blk, 0, s, nd, pt, ps, op->nfar, nq, nkc,
                               op->kappa, op->mix, op->d_coupling_lo.as<bf16x2>());
        IGB_HIP(hipGetLastError());
    }
    for (M2LChunks* c : {&op->chunks, &op->chunks_mfma}) {
        if ((st = upload(c->d_tgt, c->tgt.data(), c->tgt.size(), acct))) return st;
        if ((st = upload(c->d_pair, c->pair.data(), c->pair.size(), acct))) return st;
        if ((st = upload(c->d_len, c->len.data(), c->len.size(), acct))) return st;
        if ((st = upload(c->d_tgt_ptr, c->tgt_ptr.data(), c->tgt_ptr.size(), acct))) return st;
    }
    IGB_HIP(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    op->t_assembly_far = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return IGB_OK;
}

// Matvec work buffers of an operator for ncol columns, in bytes (0: not used):
// cluster moments x^ / y^ (and the raw hard coupling results), coupling
// partials of the vector and matrix-core paths, rounded source vectors, the
// fp32 near-product columns of bf16 operators, the S^2 far-field result and
// glued input, and the leaves' B-spline windows.
WorkSizes work_sizes(const igb_op_s* op, int ncol) {
    WorkSizes w{};
    const size_t C = size_t(ncol), nq = size_t(op->nq);
    const bool hard = op->bc == IGB_HARD;
    const size_t kinds = hard ? 3 : 1, nvec = hard ? 10 : 1;
    w.b[WorkSizes::XHAT] = C * kinds * op->nclusters * nq * sizeof(double2);
    w.b[WorkSizes::YHAT] = w.b[WorkSizes::XHAT];
    w.b[WorkSizes::YRAW] = hard ? C * nvec * op->nclusters * nq * sizeof(double2) : 0;
    w.b[WorkSizes::PART] = C * std::max<size_t>(1, op->chunks.len.size()) * nvec * nq * sizeof(double2);
    if (op->prm.precision != IGB_FP64 || mf_fp64(const_cast<igb_op>(op))) {
        const size_t ncolp = (C + 15) / 16 * 16;
        const size_t pt = op->prm.precision == IGB_FP64 ? sizeof(double2) : sizeof(float2);
        igb_op o = const_cast<igb_op>(op);
        w.b[WorkSizes::XLO] = size_t(op->nclusters) * (hard ? 7 : 1) * ncolp * lo_kbp(o) * lo_esz(o);
        w.b[WorkSizes::PART_LO] = C * std::max<size_t>(1, op->chunks_mfma.len.size()) * nvec * nq * pt;
    }
    if (op->prm.far_on_the_fly && hard && C >= size_t(MF64_MIN_COLS)) {
        // fp64 source vectors of the on-the-fly matrix-core coupling (the rounded
        // copy's buffer, shared: the two products never run in one matvec)
        const size_t ncolp = (C + 15) / 16 * 16;
        w.b[WorkSizes::XLO] = std::max(w.b[WorkSizes::XLO], size_t(op->nclusters) * 7 * ncolp * kbp_f64(op->nq) *
                                                               sizeof(double2));
    }
    if (op->prm.precision == IGB_MIX_BF16 && op->nnz > 0)
        w.b[WorkSizes::XNEAR_LO] = (C + 15) / 16 * 16 * op->N * sizeof(float2);
    if (op->nnz > 0 && ((op->prm.precision == IGB_FP64 && C >= size_t(MF64_MIN_COLS)) ||
                        op->prm.precision == IGB_MIX_FP32))
        w.b[WorkSizes::XNEAR64] = (C + 15) / 16 * 16 * op->N * sizeof(double2);
    w.b[WorkSizes::X2] = hard ? C * op->geom->n2 * sizeof(double2) : 0;   // S^0 -> S^2 copy of x
    const size_t win = (size_t(1) << op->d) + op->geom->p;
    w.b[WorkSizes::LEAFBUF] = C * kinds * clusters_on_level(op->geom->npatch, op->L) * win * win * sizeof(double2);
    return w;
}

static igb::DevBuf* work_buf(igb_op op, int i) {
    igb::DevBuf* bufs[WorkSizes::COUNT] = {&op->d_xhat, &op->d_yhat, &op->d_yraw,  &op->d_part, &op->d_xlo,
                                           &op->d_part_lo, &op->d_xnear_lo, &op->d_x2,
                                           &op->d_leafbuf, &op->d_xnear64};
    return bufs[i];
}

igb_status alloc_work(igb_op op, int ncol) {
    size_t* acct = &op->dev_bytes;
    igb_status st;
    if (!op->d_cluoff.ptr) {
        // cluster offsets are needed on the device by the tree kernels
        if ((st = upload(op->d_cluoff, op->clu_off.data(), op->clu_off.size(), acct))) return st;
    }
    if (ncol <= op->work_cols) return IGB_OK;
    const WorkSizes w = work_sizes(op, ncol);
    // the budget check covers the whole growth before anything is released
    size_t held = 0;
    for (int i = 0; i < WorkSizes::COUNT; ++i) held += work_buf(op, i)->bytes;
    igb_ctx ctx = op->geom->ctx;
    if (ctx->budget != 0 && w.total() > held && ctx->used.load() + (w.total() - held) > ctx->budget) {
        set_error("h2_matvec: HBM budget exceeded by the work vectors of %d columns (%zu held + %zu > %zu bytes)",
                  ncol, ctx->used.load(), w.total() - held, ctx->budget);
        return IGB_ERR_BUDGET;
    }
    op->clear_graphs();   // captured launches refer to the buffers released here
    op->work_cols = 0;    // until every buffer is in place
    for (int i = 0; i < WorkSizes::COUNT; ++i) {
        igb::DevBuf* b = work_buf(op, i);
        *acct -= std::min(*acct, b->bytes);
        b->release();
    }
    for (int i = 0; i < WorkSizes::COUNT; ++i)
        if (w.b[i] && (st = alloc(*work_buf(op, i), w.b[i], acct))) return st;
    op->work_cols = ncol;
    return IGB_OK;
}

igb_status timer_mark(igb_op op, int slot, hipStream_t s) {
    if (!op->profile) return IGB_OK;
    KernelTimer& t = op->timers[slot];
    if (t.used == t.pool.size()) {
        hipEvent_t e;
        IGB_HIP(hipEventCreate(&e));
        t.pool.push_back(e);
    }
    IGB_HIP(hipEventRecord(t.pool[t.used++], s));
    return IGB_OK;
}

// fp64 sound-hard coupling on the fly for blocks of >= 16 columns: the source
// vectors rounded (to fp64: copied) into the matrix-core layout, then one
// workgroup of ceil(nq / 16) waves (twice that where the products are split)
// per (chunk, 16 columns)
static void launch_m2l_otf_mfma_hard(igb_op op, const MatvecWork& W, const double2* xh, int64_t ks, int ncol,
                                     hipStream_t s) {
    const M2LChunks& C = op->chunks;
    const int64_t nchunk = int64_t(C.len.size());
    const int ncolp = (ncol + 15) / 16 * 16, nq = op->nq, kbp = kbp_f64(nq);
    double2* xv = static_cast<double2*>(W.xlo);
    const int64_t nv = op->nclusters * 7 * ncolp * kbp;
    hipLaunchKernelGGL((round_vectors<7, double2>), dim3(unsigned((nv + 255) / 256)), dim3(256), 0, s, xh, ks,
                       op->d_nodes.as<double>(), op->nclusters, nq, kbp, ncol, ncolp, xv);
    const dim3 grid(unsigned(nchunk), unsigned(ncolp / 16));
    // (an even number of row tiles splits each tile's products over two waves,
    // balanced over the 4 SIMDs of a CU)
#define IGB_OTF_MF(NWV, SLABV, SPLITV)                                                                             \
    hipLaunchKernelGGL((m2l_otf_mfma_hard<NWV, SLABV, SPLITV>), grid, dim3(64 * NWV * (SPLITV ? 2 : 1)), 0, s,      \
                       op->d_nodes.as<double>(), xv, kbp, ncolp, op->d_far_src.as<int>(), C.d_tgt.as<int>(),      \
                       C.d_pair.as<int64_t>(), C.d_len.as<int>(), nchunk, nq, ncol, op->kappa, W.part)
    switch ((nq + 15) / 16) {
        case 1: IGB_OTF_MF(1, 16, false); break;
        case 2: IGB_OTF_MF(2, 16, true); break;
        case 3: IGB_OTF_MF(3, 16, false); break;
        case 4: IGB_OTF_MF(4, 16, true); break;
        case 5: IGB_OTF_MF(5, 16, false); break;
        case 6: IGB_OTF_MF(6, 16, true); break;
        case 7: IGB_OTF_MF(7, 8, false); break;
        default: IGB_OTF_MF(8, 8, false); break;
    }
#undef IGB_OTF_MF
}

// vector path (fp64 couplings): the soft kernel keeps 8 accumulators per lane,
// the hard one 10 per column
template <int NT>
static void launch_m2l_fp64(igb_op op, const MatvecWork& W, double2* xh, int64_t ks, int ncol, hipStream_t s) {
    const double2* coup = op->d_coupling.as<double2>();
    const M2LChunks& C = op->chunks;
    const int64_t nchunk = int64_t(C.len.size());
    if (nchunk == 0) return;
    if (op->prm.far_on_the_fly) {
        const double* nd = op->d_nodes.as<double>();
        if (op->bc == IGB_HARD && ncol >= MF64_MIN_COLS) {
            launch_m2l_otf_mfma_hard(op, W, xh, ks, ncol, s);
        } else if (op->bc == IGB_HARD) {
            constexpr int RB = 4;
            hipLaunchKernelGGL((m2l_otf_hard<NT, RB>), dim3(unsigned(nchunk), unsigned((ncol + RB - 1) / RB)),
                               dim3(NT), 0, s, nd, xh, ks, op->d_far_src.as<int>(), C.d_tgt.as<int>(),
                               C.d_pair.as<int64_t>(), C.d_len.as<int>(), nchunk, op->nq, ncol, op->kappa,
                               W.part);
        } else if (ncol >= 16) {
            // (16 accumulators per lane: each kernel value serves twice the columns;
            // 4.6 -> 3.4 ms at 16 columns on the level-6 star, slower for one column)
            constexpr int RB = 16;
            hipLaunchKernelGGL((m2l_otf_soft<NT, RB>), dim3(unsigned(nchunk), unsigned((ncol + RB - 1) / RB)),
                               dim3(NT), 0, s, nd, xh, op->d_far_src.as<int>(), C.d_tgt.as<int>(),
                               C.d_pair.as<int64_t>(), C.d_len.as<int>(), nchunk, op->nq, ncol, op->kappa, op->mix,
                               W.part);
        } else {
            constexpr int RB = 8;
            hipLaunchKernelGGL((m2l_otf_soft<NT, RB>), dim3(unsigned(nchunk), unsigned((ncol + RB - 1) / RB)),
                               dim3(NT), 0, s, nd, xh, op->d_far_src.as<int>(), C.d_tgt.as<int>(),
                               C.d_pair.as<int64_t>(), C.d_len.as<int>(), nchunk, op->nq, ncol, op->kappa, op->mix,
                               W.part);
        }
        return;
    }
    if (op->bc == IGB_HARD) {
        constexpr int RB = 2;
        hipLaunchKernelGGL((m2l_hard_chunks<NT, double2, RB>), dim3(unsigned(nchunk), unsigned((ncol + RB - 1) / RB)),
                           dim3(NT), 0, s, coup, xh, ks, op->d_nodes.as<double>(), op->d_far_src.as<int>(),
                           C.d_pair.as<int64_t>(), C.d_len.as<int>(), nchunk, op->nq, ncol, W.part);
    } else if (ncol == 1 && op->d_lr.ptr) {
        hipLaunchKernelGGL(m2l_chunks_lowrank<LR_WAVES>, dim3(unsigned(nchunk)), dim3(64 * LR_WAVES), 0, s,
                           op->d_lr.as<double2>(),
                           op->d_lr_rank.as<int>(), op->d_lr_off.as<int64_t>(), xh, op->d_far_src.as<int>(),
                           C.d_pair.as<int64_t>(), C.d_len.as<int>(), nchunk, op->nq, W.part);
    } else if (ncol == 1 && op->nq <= 64) {
        hipLaunchKernelGGL(m2l_chunks_wave, dim3(unsigned(nchunk)), dim3(64), 0, s, coup, xh, op->d_far_src.as<int>(),
                           C.d_pair.as<int64_t>(), C.d_len.as<int>(), nchunk, op->nq, W.part);
    } else if (ncol == 1) {
        hipLaunchKernelGGL((m2l_chunks<NT, double2, 1>), dim3(unsigned(nchunk), 1u), dim3(NT), 0, s, coup, xh,
                           op->d_far_src.as<int>(), C.d_pair.as<int64_t>(), C.d_len.as<int>(), nchunk, op->nq, ncol,
                           W.part);
    } else {
        constexpr int RB = 8;
        hipLaunchKernelGGL((m2l_chunks<NT, double2, RB>), dim3(unsigned(nchunk), unsigned((ncol + RB - 1) / RB)),
                           dim3(NT), 0, s, coup, xh, op->d_far_src.as<int>(), C.d_pair.as<int64_t>(), C.d_len.as<int>(),
                           nchunk, op->nq, ncol, W.part);
    }
}

// matrix-core path (reduced-precision couplings)
template <class OPS, bool HARD>
static void launch_m2l_lo_t(igb_op op, const MatvecWork& W, const double2* xh, int64_t ks, int ncol, hipStream_t s) {
    using LT = typename OPS::LT;
    const M2LChunks& C = op->chunks_mfma;
    const int64_t nchunk = int64_t(C.len.size());
    const int ncolp = (ncol + 15) / 16 * 16, kbp = lo_kbp(op), nq = op->nq;
    const int64_t nv = op->nclusters * (HARD ? 7 : 1) * ncolp * kbp;
    hipLaunchKernelGGL((round_vectors<HARD ? 7 : 1, LT>), dim3(unsigned((nv + 255) / 256)), dim3(256), 0, s, xh, ks,
                       op->d_nodes.as<double>(), op->nclusters, nq, kbp, ncol, ncolp, static_cast<LT*>(W.xlo));
    (void)timer_mark(op, 0, s);
    using PT = typename OPS::PT;
    const LT* cp = op->prm.precision == IGB_FP64 ? op->d_coupling.as<LT>() : op->d_coupling_lo.as<LT>();
    if (!HARD && nchunk > 0) {
        const dim3 grid(unsigned(nchunk), unsigned(ncolp / 16));
        const LT* xp = static_cast<LT*>(W.xlo);
        PT* pp = static_cast<PT*>(W.part_lo);
#define IGB_SOFT_MT(MTV)                                                                                          \
    hipLaunchKernelGGL((m2l_mfma_soft<OPS, MTV>), grid, dim3(256), 0, s, cp, lo_nkc(op), xp, kbp, ncolp,           \
                       op->d_far_src.as<int>(), C.d_pair.as<int64_t>(), C.d_len.as<int>(), nchunk, nq, ncol, pp)
        switch ((nq + 15) / 16) {
            case 1: IGB_SOFT_MT(1); break;
            case 2: IGB_SOFT_MT(2); break;
            case 3: IGB_SOFT_MT(3); break;
            case 4: IGB_SOFT_MT(4); break;
            case 5: IGB_SOFT_MT(5); break;
            case 6: IGB_SOFT_MT(6); break;
            case 7: IGB_SOFT_MT(7); break;
            default: IGB_SOFT_MT(8); break;
        }
#undef IGB_SOFT_MT
    } else if (nchunk > 0) {
        // fp64 accumulators are twice the size: one row tile per wave
        constexpr int RPWO = std::is_same<OPS, MfmaF64>::value ? 1 : M2L_RPW;
        hipLaunchKernelGGL((m2l_mfma<OPS, HARD, RPWO>), dim3(unsigned(nchunk), unsigned(ncolp / 16)),
                           dim3(64 * (((nq + 15) / 16 + RPWO - 1) / RPWO)), 0, s, cp, lo_nkc(op),
                           static_cast<LT*>(W.xlo), kbp, ncolp, op->d_far_src.as<int>(), C.d_pair.as<int64_t>(),
                           C.d_len.as<int>(), nchunk, nq, ncol, static_cast<PT*>(W.part_lo));
    }
    (void)timer_mark(op, 0, s);
}

// fp64 sound-soft blocks of >= 16 columns: up to 4 column tiles per wave
static void launch_m2l_f64_soft(igb_op op, const MatvecWork& W, const double2* xh, int ncol, hipStream_t s) {
    const M2LChunks& C = op->chunks_mfma;
    const int64_t nchunk = int64_t(C.len.size());
    const int ncolp = (ncol + 15) / 16 * 16, kbp = lo_kbp(op), nq = op->nq;
    const int64_t nv = op->nclusters * ncolp * kbp;
    double2* xlo = static_cast<double2*>(W.xlo);
    hipLaunchKernelGGL((round_vectors<1, double2>), dim3(unsigned((nv + 255) / 256)), dim3(256), 0, s, xh, int64_t(0),
                       op->d_nodes.as<double>(), op->nclusters, nq, kbp, ncol, ncolp, xlo);
    (void)timer_mark(op, 0, s);
    if (nchunk > 0) {
        // NC column tiles per workgroup, NC dividing the padded tile count (the
        // last workgroup's tiles stay inside the rounded source vectors)
        // (the widest grouping that keeps at least 512 workgroups, 2 per CU: on
        // the level-5 sphere the tuner's choice at 32 and 64 columns)
        const int ntile = ncolp / 16;
        int nc = 1;
        for (int c : {4, 2})
            if (ntile % c == 0 && nchunk * (ntile / c) >= 512) {
                nc = c;
                break;
            }
        if (op->tile_m2l_nc > 0 && ntile % op->tile_m2l_nc == 0) nc = op->tile_m2l_nc;   // tuned shape
        const dim3 grid(unsigned(nchunk), unsigned((ntile + nc - 1) / nc)), block(64 * ((nq + 15) / 16));
        const double2* cp = op->d_coupling.as<double2>();
        double2* pp = static_cast<double2*>(W.part_lo);
        const int* fs = op->d_far_src.as<int>();
        const int64_t* cpair = C.d_pair.as<int64_t>();
        const int* clen = C.d_len.as<int>();
        if (nc == 4)
            hipLaunchKernelGGL((m2l_mfma64_soft<4, 1>), grid, block, 0, s, cp, lo_nkc(op), xlo, kbp, ncolp, fs, cpair,
                               clen, nchunk, nq, ncol, pp);
        else if (nc == 2)
            hipLaunchKernelGGL((m2l_mfma64_soft<2, 2>), grid, block, 0, s, cp, lo_nkc(op), xlo, kbp, ncolp, fs, cpair,
                               clen, nchunk, nq, ncol, pp);
        else
            hipLaunchKernelGGL((m2l_mfma64_soft<1, 4>), grid, block, 0, s, cp, lo_nkc(op), xlo, kbp, ncolp, fs, cpair,
                               clen, nchunk, nq, ncol, pp);
    }
    (void)timer_mark(op, 0, s);
}

// coupling partials [chunk][nvec][nq][ncol] of the far pairs.  kind: 0 fp64
// partials of the vector path, 1 fp32 partials of the matrix-core path at
// reduced precision, 2 fp64 partials of the matrix-core path
static igb_status launch_m2l(igb_op op, const MatvecWork& W, double2* xh, int64_t ks, bool low, int ncol, hipStream_t s, int& kind) {
    const bool lo = low && op->prm.precision != IGB_FP64;
    const bool hard = op->bc == IGB_HARD;
    // fp64: the matrix cores pay off for blocks of at least MF64_MIN_COLS
    // columns; a single column is HBM-bound on the vector path
    kind = lo ? 1 : (mf_fp64(op) && ncol >= MF64_MIN_COLS) ? 2 : 0;
    if (kind == 2) {
        if (hard) launch_m2l_lo_t<MfmaF64, true>(op, W, xh, ks, ncol, s);
        else launch_m2l_f64_soft(op, W, xh, ncol, s);
    } else if (!lo) {
        if ((op->nq + 63) / 64 * 64 > 128) {
            set_error("h2_matvec: interpolation degree too large for the coupling kernel");
            return IGB_ERR_ARG;
        }
        igb_status st;
        if ((st = timer_mark(op, 0, s))) return st;
        if (op->nq <= 64) launch_m2l_fp64<64>(op, W, xh, ks, ncol, s);
        else launch_m2l_fp64<128>(op, W, xh, ks, ncol, s);
        if ((st = timer_mark(op, 0, s))) return st;
    } else if (op->prm.precision == IGB_MIX_FP32) {
        if (hard) launch_m2l_lo_t<MfmaF32, true>(op, W, xh, ks, ncol, s);
        else launch_m2l_lo_t<MfmaF32, false>(op, W, xh, ks, ncol, s);
    } else {
        if (hard) launch_m2l_lo_t<MfmaBf16, true>(op, W, xh, ks, ncol, s);
        else launch_m2l_lo_t<MfmaBf16, false>(op, W, xh, ks, ncol, s);
    }
    IGB_HIP(hipGetLastError());
    return IGB_OK;
}

static inline unsigned blocks_for(int64_t n, int t) { return unsigned((n + t - 1) / t); }

static igb_status matvec_launches(igb_op op, const MatvecWork& W, const double* x, double* y, int ncol, int parts,
                                  hipStream_t s);

// y = A x: the launch sequence is captured once per (x, y, columns, parts,
// stream) into a HIP graph and replayed; it holds kernel launches only (no
// memsets, no allocation).  Kernel timing (profile mode) launches directly.
// leaf moments of one kind (derivative flags du, dv) of ncol columns into xh
static void launch_leaf_moments(igb_op op, const double2* x2, double2* xh, int du, int dv, int ncol, hipStream_t s) {
    igb_geom g = op->geom;
    const int q = op->q, L = op->L, nq = op->nq;
    const int64_t nleaf = clusters_on_level(g->npatch, L);
    const int w = (1 << op->d) + g->p;
    const int64_t stride_kind = int64_t(1 << L) * (q + 1) * w;
    if (w <= LM_W)
        hipLaunchKernelGGL(leaf_moments_wg, dim3(unsigned(nleaf), unsigned(ncol)), dim3(64), 0, s, x2, g->n2,
                           op->d_m1.as<double>(), q, op->d, g->p, L, g->k, op->clu_off[L], xh, du, dv, stride_kind,
                           ncol);
    else
        hipLaunchKernelGGL(leaf_moments, dim3(blocks_for(nleaf * nq * ncol, 256)), dim3(256), 0, s, x2, g->n2,
                           op->d_m1.as<double>(), q, op->d, g->p, L, g->k, op->clu_off[L], nleaf, xh, du, dv,
                           stride_kind, ncol);
}

// y += c t over n complex entries
__global__ void caxpy(double2* __restrict__ y, const double2* __restrict__ t, double2 c, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) y[i] = cfma(c, t[i], y[i]);
}

// Lazy sum of separately stored H^2 matrices: y = A_0 x, then y += c_i (A_i x) in order
static igb_status matvec_sum(igb_op op, const double* x, double* y, int ncol, int parts, hipStream_t s) {
    igb_status st;
    const int64_t n = int64_t(ncol) * op->N;
    if (op->sum_coef.front().x != 1.0 || op->sum_coef.front().y != 0.0) {
        set_error("h2_matvec: the first part of a lazy sum must have coefficient 1");
        return IGB_ERR_ARG;
    }
    if ((st = matvec_device(op->sum_parts.front(), x, y, ncol, parts, s))) return st;
    if (op->sum_parts.size() < 2) return IGB_OK;
    // grows with the column count; freed with the operator
    if ((st = op_reserve(op, op->d_sum_tmp, size_t(n) * sizeof(double2), "h2_matvec"))) return st;
    double2* t = op->d_sum_tmp.as<double2>();
    for (size_t i = 1; i < op->sum_parts.size(); ++i) {
        if ((st = matvec_device(op->sum_parts[i], x, reinterpret_cast<double*>(t), ncol, parts, s))) return st;
        hipLaunchKernelGGL(caxpy, dim3(blocks_for(n, 256)), dim3(256), 0, s, reinterpret_cast<double2*>(y), t,
                           op->sum_coef[i], n);
        IGB_HIP(hipGetLastError());
    }
    return IGB_OK;
}

// the operator's own work buffers
static MatvecWork own_work(igb_op op) {
    MatvecWork W;
    W.xhat = op->d_xhat.as<double2>();
    W.yhat = op->d_yhat.as<double2>();
    W.yraw = op->d_yraw.as<double2>();
    W.part = op->d_part.as<double2>();
    W.xlo = op->d_xlo.ptr;
    W.part_lo = op->d_part_lo.ptr;
    W.xnear_lo = op->d_xnear_lo.as<float2>();
    W.x2 = op->d_x2.as<double2>();
    W.leafbuf = op->d_leafbuf.as<double2>();
    W.xnear64 = op->d_xnear64.as<double2>();
    return W;
}

// ---------------------------------------------------------------------------
// Work buffers without allocation: one file-scope device array per GPU.  In
// host code `scratch` names a host-side stand-in, so host code uses only the
// device address that hipGetSymbolAddress returned for the current device,
// taken once per device at context creation (scratch_init).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[IGB_NOALLOC_SCRATCH_BYTES];
static std::mutex scratch_mu;
static void* scratch_dev[SCRATCH_MAX_DEVICES];

igb_status scratch_init(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) {
        set_error("igb_ctx_create: device %d beyond the %d devices the matvec scratch supports", device,
                  SCRATCH_MAX_DEVICES);
        return IGB_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (scratch_dev[device]) return IGB_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));   // device `device` is current
    if (e != hipSuccess || !ptr) {
        set_error("igb_ctx_create: hipGetSymbolAddress of the matvec scratch failed: %s", hipGetErrorString(e));
        return IGB_ERR_HIP;
    }
    scratch_dev[device] = ptr;
    return IGB_OK;
}

igb_status matvec_noalloc(igb_op op, const double* x, double* y, int ncol, int parts, hipStream_t s) {
    const int dev = op->geom->ctx->device;
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(scratch_mu);
        base = dev >= 0 && dev < SCRATCH_MAX_DEVICES ? scratch_dev[dev] : nullptr;
    }
    if (!base) {
        set_error("h2_matvec_noalloc: no scratch address for device %d (context not created on it)", dev);
        return IGB_ERR_ARG;
    }
    if (!op->d_cluoff.ptr) {
        set_error("h2_matvec_noalloc: operator not assembled on the device");
        return IGB_ERR_ARG;
    }
    // carve the work buffers out of the scratch, each 256-byte aligned
    const WorkSizes w = work_sizes(op, ncol);
    size_t off[WorkSizes::COUNT], end = 0;
    for (int i = 0; i < WorkSizes::COUNT; ++i) {
        off[i] = end;
        end += (w.b[i] + 255) / 256 * 256;
    }
    if (end > IGB_NOALLOC_SCRATCH_BYTES) {
        set_error("h2_matvec_noalloc: %d columns need %zu bytes of work buffers, more than the %zu-byte scratch",
                  ncol, end, size_t(IGB_NOALLOC_SCRATCH_BYTES));
        return IGB_ERR_ARG;
    }
    unsigned char* b = static_cast<unsigned char*>(base);
    auto at = [&](int i) -> void* { return w.b[i] ? static_cast<void*>(b + off[i]) : nullptr; };
    MatvecWork W;
    W.xhat = static_cast<double2*>(at(WorkSizes::XHAT));
    W.yhat = static_cast<double2*>(at(WorkSizes::YHAT));
    W.yraw = static_cast<double2*>(at(WorkSizes::YRAW));
    W.part = static_cast<double2*>(at(WorkSizes::PART));
    W.xlo = at(WorkSizes::XLO);
    W.part_lo = at(WorkSizes::PART_LO);
    W.xnear_lo = static_cast<float2*>(at(WorkSizes::XNEAR_LO));
    W.x2 = static_cast<double2*>(at(WorkSizes::X2));
    W.leafbuf = static_cast<double2*>(at(WorkSizes::LEAFBUF));
    W.xnear64 = static_cast<double2*>(at(WorkSizes::XNEAR64));
    return matvec_launches(op, W, x, y, ncol, parts, s);
}

igb_status matvec_device(igb_op op, const double* x, double* y, int ncol, int parts, hipStream_t s) {
    igb_status st;
    if (!op->sum_parts.empty()) return matvec_sum(op, x, y, ncol, parts, s);
    if ((st = alloc_work(op, ncol))) return st;
    const MatvecWork W = own_work(op);
    if (!op->use_graphs || op->profile || s == nullptr) return matvec_launches(op, W, x, y, ncol, parts, s);
    const igb_op_s::GraphKey key{x, y, ncol, parts, s};
    for (auto& gr : op->graphs)
        if (gr.first == key) {
            IGB_HIP(hipGraphLaunch(gr.second, s));
            return IGB_OK;
        }
    if (op->graphs.size() >= 512) op->clear_graphs();
    hipGraph_t graph = nullptr;
    IGB_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    st = matvec_launches(op, W, x, y, ncol, parts, s);
    const hipError_t ce = hipStreamEndCapture(s, &graph);
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (ce != hipSuccess) {
        set_error("h2_matvec: graph capture failed: %s", hipGetErrorString(ce));
        return IGB_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
        set_error("h2_matvec: graph instantiation failed: %s", hipGetErrorString(ie));
        return IGB_ERR_HIP;
    }
    op->graphs.emplace_back(key, exec);
    IGB_HIP(hipGraphLaunch(exec, s));
    return IGB_OK;
}

static igb_status matvec_launches(igb_op op, const MatvecWork& W, const double* x, double* y, int ncol, int parts,
                                  hipStream_t s) {
    const bool low = (parts & IGB_MV_LOWPREC) != 0;
    igb_status st;
    igb_geom g = op->geom;
    const int q = op->q, nq = op->nq, L = op->L;
    const bool hard = op->bc == IGB_HARD;
    const double2* X = reinterpret_cast<const double2*>(x);
    double2* Y = reinterpret_cast<double2*>(y);
    double2* xh = W.xhat;
    double2* yh = W.yhat;
    const int64_t N = op->N;
    const bool far = (parts & IGB_PART_FAR) && op->nfar > 0;
    if (far) {
        const double2* x2 = X;
        if (hard) {
            hipLaunchKernelGGL(glue_gather, dim3(blocks_for(g->n2 * ncol, 256)), dim3(256), 0, s,
                               op->d_s2_to_s0.as<int>(), X, N, W.x2, g->n2, ncol);
            x2 = W.x2;
        }
        const int kinds = hard ? 3 : 1;
        const int64_t ks = op->nclusters * nq * ncol;  // stride between moment kinds
        const int du[3] = {0, 1, 0}, dv[3] = {0, 0, 1};
        const int64_t nleaf = clusters_on_level(g->npatch, L);
        const int64_t stride_kind = int64_t(1 << L) * (q + 1) * ((1 << op->d) + g->p);
        if ((st = timer_mark(op, 2, s))) return st;
        for (int kd = 0; kd < kinds; ++kd) {
            launch_leaf_moments(op, x2, xh + kd * ks, du[kd], dv[kd], ncol, s);
            launch_m2m_levels(op->d_T.as<double>(), q, L, g->npatch, op->clu_off, xh + kd * ks, ncol, s,
                              op->far_lmin);
        }
        if ((st = timer_mark(op, 2, s))) return st;
        int pkind = 0;
        if ((st = launch_m2l(op, W, xh, ks, low, ncol, s, pkind))) return st;
        if ((st = timer_mark(op, 3, s))) return st;
        const int nvec = hard ? 10 : 1;
        double2* red_out = W.yraw;
        const int64_t per = int64_t(nvec) * nq * ncol;
        if (!hard) {
            // sound-soft: the downward kernel sums the chunk partials itself
        } else if (pkind == 1)
            hipLaunchKernelGGL(m2l_reduce<float2>, dim3(blocks_for(op->nclusters * per, 256)), dim3(256), 0, s,
                               static_cast<float2*>(W.part_lo), op->chunks_mfma.d_tgt_ptr.as<int>(), op->nclusters, per,
                               red_out);
        else if (pkind == 2)
            hipLaunchKernelGGL(m2l_reduce<double2>, dim3(blocks_for(op->nclusters * per, 256)), dim3(256), 0, s,
                               static_cast<double2*>(W.part_lo), op->chunks_mfma.d_tgt_ptr.as<int>(), op->nclusters, per,
                               red_out);
        else
            hipLaunchKernelGGL(m2l_reduce<double2>, dim3(blocks_for(op->nclusters * per, 256)), dim3(256), 0, s,
                               W.part, op->chunks.d_tgt_ptr.as<int>(), op->nclusters, per, red_out);
        if (hard)
            hipLaunchKernelGGL(m2l_finalize_hard, dim3(blocks_for(op->nclusters * nq * ncol, 256)), dim3(256), 0, s,
                               W.yraw, op->d_nodes.as<double>(), op->nclusters, nq, op->kappa,
                               op->hmix, ks, ncol, yh);
        const int w = (1 << op->d) + g->p;
        size_t dlds = 0;
        const int dcb = down_cols(ncol, q + 1, w, dlds);
        const dim3 dgrid(unsigned(nleaf), unsigned((ncol + dcb - 1) / dcb)), dblock(dcb >= 4 ? 256 : TREE_THREADS);
        const double* Tc = op->d_Tc.as<double>();
        const int64_t* cof = op->d_cluoff.as<int64_t>();
        const double* m1 = op->d_m1.as<double>();
        double2* lb = W.leafbuf;
        const int lmin = op->far_lmin;
        if (hard) {
            for (int kd = 0; kd < kinds; ++kd)
                hipLaunchKernelGGL(down_project_leaf<double2>, dgrid, dblock, dlds, s, yh + kd * ks,
                                   static_cast<const double2*>(nullptr), static_cast<const int*>(nullptr), Tc, cof, m1,
                                   q, w, L, lmin, du[kd], dv[kd], stride_kind, ncol, dcb,
                                   lb + kd * nleaf * ncol * w * w);
        } else if (pkind == 1) {
            hipLaunchKernelGGL(down_project_leaf<float2>, dgrid, dblock, dlds, s, yh, static_cast<float2*>(W.part_lo),
                               op->chunks_mfma.d_tgt_ptr.as<int>(), Tc, cof, m1, q, w, L, lmin, 0, 0, stride_kind,
                               ncol, dcb, lb);
        } else {
            const bool lo = pkind == 2;
            hipLaunchKernelGGL(down_project_leaf<double2>, dgrid, dblock, dlds, s, yh,
                               lo ? static_cast<double2*>(W.part_lo) : W.part,
                               (lo ? op->chunks_mfma : op->chunks).d_tgt_ptr.as<int>(), Tc, cof, m1, q, w, L, lmin,
                               0, 0, stride_kind, ncol, dcb, lb);
        }
        if ((st = timer_mark(op, 3, s))) return st;
    }
    if ((st = timer_mark(op, 1, s))) return st;
    // the far part: gathered from the downward pass's leaf buffers by the near kernels
    const FarLeaves yfar{far ? W.leafbuf : nullptr, op->d, g->p, op->L, g->k, g->npatch, hard ? 3 : 1, ncol};
    const int* s0p = hard ? op->d_s0_ptr.as<int>() : nullptr;
    const int* s0r = hard ? op->d_s0_reps.as<int>() : nullptr;
    const int use_near = (parts & IGB_PART_NEAR) ? 1 : 0;
    const dim3 sg(blocks_for(N * 64, 256)), sb(256);
    const int64_t* rp = op->d_rowptr.as<int64_t>();
    const int64_t* rco = op->d_row_coff.as<int64_t>();
    const int* dcl = op->d_dcol.as<int>();
    const double2* vl = op->d_val.as<double2>();
    if (low && op->d_val_lo.ptr) {
        const int ncb = (ncol + 15) / 16;
        float2* xt = W.xnear_lo;
        if (use_near)
            hipLaunchKernelGGL(round_columns_t, dim3(blocks_for(int64_t(ncb) * N * 16, 256)), dim3(256), 0, s, X, N,
                               ncol, ncb, xt);
        hipLaunchKernelGGL(near_tiles_mfma, dim3(unsigned(op->near_tiles.size()), unsigned(ncb)),
                           dim3(64 * NEAR_TILE_WAVES), 0, s,
                           op->d_near_tiles.as<NearTile>(), int64_t(op->near_tiles.size()),
                           op->d_near_tile_cols.as<int>(),
                           op->d_val_lo.as<float2>(), xt, N, yfar, s0p, s0r, use_near, ncol, Y);
    } else if (op->d_val64.ptr && W.xnear64 &&
               (op->prm.precision == IGB_FP64 ? ncol >= MF64_MIN_COLS : low)) {
        // fp64 matrix cores over the tiles: columns transposed into 16-wide rows once
        const int ncb = (ncol + 15) / 16;
        if (use_near)
            hipLaunchKernelGGL(columns_t64, dim3(blocks_for(int64_t(ncb) * N * 16, 256)), dim3(256), 0, s, X, N,
                               ncol, ncb, W.xnear64);
        // NC column tiles per workgroup (each tile value read serves 16 NC columns):
        // 2 when it divides the column tile count and the grid keeps at least
        // 512 workgroups (2 per CU), else 1 (4 measured slower on the level-5
        // sphere and the level-6 star); the column results do not depend on NC
        const int64_t ntl0 = int64_t(op->near_tiles.size());
        int nct = ncb % 2 == 0 && ntl0 * (ncb / 2) >= 512 ? 2 : 1;
        if (op->tile_near_nct > 0 && ncb % op->tile_near_nct == 0) nct = op->tile_near_nct;   // tuned shape
        const dim3 tg(unsigned(op->near_tiles.size()), unsigned(ncb / nct)), tb(64 * NEAR64_WAVES);
        const NearTile* tl = op->d_near_tiles.as<NearTile>();
        const int64_t ntl = int64_t(op->near_tiles.size());
        const int* tcl = op->d_near_tile_cols.as<int>();
        const double2* v64 = op->d_val64.as<double2>();
        if (nct == 4)
            hipLaunchKernelGGL(near_tiles_mfma64<4>, tg, tb, 0, s, tl, ntl, tcl, v64, W.xnear64, N, yfar, s0p,
                               s0r, use_near, ncol, Y);
        else if (nct == 2)
            hipLaunchKernelGGL(near_tiles_mfma64<2>, tg, tb, 0, s, tl, ntl, tcl, v64, W.xnear64, N, yfar, s0p,
                               s0r, use_near, ncol, Y);
        else
            hipLaunchKernelGGL(near_tiles_mfma64<1>, tg, tb, 0, s, tl, ntl, tcl, v64, W.xnear64, N, yfar, s0p,
                               s0r, use_near, ncol, Y);
    } else if (ncol == 1 && use_near && !op->near_wgs.empty() &&
               size_t(op->near_list_max) * sizeof(double2) <= size_t(g->ctx->lds_max)) {
        hipLaunchKernelGGL(spmv_groups<NEAR_GROUP_ROWS>, dim3(unsigned(op->near_wgs.size())),
                           dim3(64 * NEAR_GROUP_ROWS), size_t(op->near_list_max) * sizeof(double2), s,
                           op->d_near_wgs.as<NearGroupWG>(), op->d_near_grp_rows.as<int>(), rp, dcl, vl, X, yfar,
                           s0p, s0r, Y);
    } else if (ncol == 1) {
        hipLaunchKernelGGL(spmv_combine<1>, sg, sb, 0, s, rp, rco, dcl, vl, X, N, yfar, s0p, s0r, use_near,
                           ncol, Y);
    } else {
        hipLaunchKernelGGL(spmv_combine<4>, sg, sb, 0, s, rp, rco, dcl, vl, X, N, yfar, s0p, s0r, use_near,
                           ncol, Y);
    }
    IGB_HIP(hipGetLastError());
    if ((st = timer_mark(op, 1, s))) return st;
    return IGB_OK;
}

int smooth_order(igb_op op, int base) {
    return std::min(NGMAX, base + kd_boost(op->kd_elem) + std::max(0, op->prm.quad_extra));
}

// bytes of the right-hand side and far-field buffers for ndir directions and
// nobs observation directions (operator-owned, kept between calls)
size_t quad_buffer_bytes(const igb_op_s* op, int ndir, int nobs) {
    const igb_geom_s* g = op->geom;
    const size_t nl = size_t(g->p + 1) * (g->p + 1);
    const int nqd = smooth_order(const_cast<igb_op>(op), 6);
    const size_t npts = size_t(g->nelem) * nqd * nqd;
    return size_t(NGMAX + 1) * 2 * NGMAX * sizeof(double) + size_t(3) * ndir * sizeof(double) +
           size_t(ndir) * g->nelem * nl * sizeof(double2) + size_t(3) * nobs * sizeof(double) +
           npts * 8 * sizeof(double) + size_t(ndir) * npts * sizeof(double2);
}

// the Gauss-Legendre table on the device, once per operator
static igb_status gauss_on_device(igb_op op) {
    if (op->d_gauss.ptr) return IGB_OK;
    const std::vector<double> gl = gauss_table();
    if (igb_status st = op_reserve(op, op->d_gauss, gl.size() * sizeof(double), "gauss table")) return st;
    IGB_HIP(hipMemcpy(op->d_gauss.ptr, gl.data(), gl.size() * sizeof(double), hipMemcpyHostToDevice));
    return IGB_OK;
}

igb_status rhs_device(igb_op op, const double* dirs, int ndir, double* b, hipStream_t s) {
    igb_geom g = op->geom;
    std::vector<double> dn(3 * ndir);
    for (int i = 0; i < ndir; ++i) {
        double nr = std::sqrt(dirs[3 * i] * dirs[3 * i] + dirs[3 * i + 1] * dirs[3 * i + 1] +
                              dirs[3 * i + 2] * dirs[3 * i + 2]);
        if (!(nr >= 1e-12)) {
            set_error("cfie_rhs: direction %d has norm < 1e-12", i);
            return IGB_ERR_ARG;
        }
        for (int c = 0; c < 3; ++c) dn[3 * i + c] = dirs[3 * i + c] / nr;
    }
    igb_status st;
    // operator-owned buffers, kept between calls (no allocation or free per call
    // once they have grown): Gauss table, directions, element contributions
    const int NL = (g->p + 1) * (g->p + 1);
    if ((st = gauss_on_device(op)) || (st = op_reserve(op, op->d_q_dirs, size_t(3) * ndir * sizeof(double), "cfie_rhs")) ||
        (st = op_reserve(op, op->d_q_loc, size_t(ndir) * g->nelem * NL * sizeof(double2), "cfie_rhs")))
        return st;
    IGB_HIP(hipStreamSynchronize(s));   // earlier work on s may still read the direction buffer
    IGB_HIP(hipMemcpy(op->d_q_dirs.ptr, dn.data(), dn.size() * sizeof(double), hipMemcpyHostToDevice));
    const DevBuf& d_dirs = op->d_q_dirs;
    const DevBuf& d_loc = op->d_q_loc;
    QuadGeoArgs A{g->d_bez.as<double>(), g->d_pg.as<int>(), g->d_C1.as<double>(), op->d_gauss.as<double>(),
                  g->nel1, g->p, smooth_order(op, 6), g->nelem};
    const bool hard = op->bc == IGB_HARD;
    dim3 grid1(unsigned((g->nelem + 127) / 128), unsigned(ndir));
    dim3 grid2(unsigned((op->N + 255) / 256), unsigned(ndir));
    const igb_op sp = op->sum_parts.empty() ? op : op->sum_parts.front();   // holds the space maps
    const int* s0p = hard ? sp->d_s0_ptr.as<int>() : nullptr;
    const int* s0r = hard ? sp->d_s0_reps.as<int>() : nullptr;
    double2* B = reinterpret_cast<double2*>(b);
    if ((st = with_degree(g->p, "cfie_rhs", [&](auto deg) {
             constexpr int P = decltype(deg)::value;
             hipLaunchKernelGGL(rhs_elements<P>, grid1, dim3(128), 0, s, A, d_dirs.as<double>(), ndir, op->kappa,
                                op->rn, op->rd, d_loc.as<double2>());
             hipLaunchKernelGGL(rhs_gather<P>, grid2, dim3(256), 0, s, d_loc.as<double2>(), ndir, g->nelem,
                                g->nel1, g->k, op->N, s0p, s0r, B);
             return IGB_OK;
         })))
        return st;
    IGB_HIP(hipGetLastError());
    return IGB_OK;
}

igb_status farfield_device(igb_op op, const double* coeffs, int ndir, const double* obs, int nobs,
                           double* uinf, hipStream_t s) {
    igb_geom g = op->geom;
    std::vector<double> on(3 * nobs);
    for (int i = 0; i < nobs; ++i) {
        double nr = std::sqrt(obs[3 * i] * obs[3 * i] + obs[3 * i + 1] * obs[3 * i + 1] + obs[3 * i + 2] * obs[3 * i + 2]);
        if (!(nr >= 1e-12)) {
            set_error("farfield: observation direction %d has norm < 1e-12", i);
            return IGB_ERR_ARG;
        }
        for (int c = 0; c < 3; ++c) on[3 * i + c] = obs[3 * i + c] / nr;
    }
    igb_status st;
    const int nqd = smooth_order(op, 6);
    const int64_t npts = g->nelem * nqd * nqd;
    // operator-owned buffers, kept between calls: Gauss table, observation
    // directions, quadrature points and densities
    if ((st = gauss_on_device(op)) || (st = op_reserve(op, op->d_q_obs, on.size() * sizeof(double), "farfield")) ||
        (st = op_reserve(op, op->d_q_geo, size_t(npts) * 8 * sizeof(double), "farfield")) ||
        (st = op_reserve(op, op->d_q_dens, size_t(ndir) * npts * sizeof(double2), "farfield")))
        return st;
    IGB_HIP(hipStreamSynchronize(s));   // earlier work on s may still read these buffers
    IGB_HIP(hipMemcpy(op->d_q_obs.ptr, on.data(), on.size() * sizeof(double), hipMemcpyHostToDevice));
    const DevBuf& d_obs = op->d_q_obs;
    const DevBuf& d_geo = op->d_q_geo;
    const DevBuf& d_dens = op->d_q_dens;
    QuadGeoArgs A{g->d_bez.as<double>(), g->d_pg.as<int>(), g->d_C1.as<double>(), op->d_gauss.as<double>(),
                  g->nel1, g->p, nqd, g->nelem};
    const bool hard = op->bc == IGB_HARD;
    const double2* C = reinterpret_cast<const double2*>(coeffs);
    const igb_op sp = op->sum_parts.empty() ? op : op->sum_parts.front();   // holds the space maps
    const int* s2s0 = hard ? sp->d_s2_to_s0.as<int>() : nullptr;
    if ((st = with_degree(g->p, "farfield", [&](auto deg) {
             constexpr int P = decltype(deg)::value;
             hipLaunchKernelGGL(density_points<P>, dim3(unsigned((npts + 255) / 256)), dim3(256), 0, s, A, C,
                                ndir, op->N, s2s0, g->k, d_geo.as<double>(), d_dens.as<double2>());
             return IGB_OK;
         })))
        return st;
    hipLaunchKernelGGL(farfield_sum, dim3(unsigned(nobs), unsigned(ndir)), dim3(256), 0, s, d_geo.as<double>(),
                       d_dens.as<double2>(), npts, d_obs.as<double>(), nobs, op->kappa, hard ? 1 : 0,
                       reinterpret_cast<double2*>(uinf));
    IGB_HIP(hipGetLastError());
    IGB_HIP(hipStreamSynchronize(s));
    return IGB_OK;
}

igb_status potential_device(igb_op op, const double* coeffs, int ndir, const double* points, int npt, double* u,
                            hipStream_t s) {
    igb_geom g = op->geom;
    for (int i = 0; i < 3 * npt; ++i)
        if (!std::isfinite(points[i])) {
            set_error("potential: point %d is not finite", i / 3);
            return IGB_ERR_ARG;
        }
    igb_status st;
    const int nqd = smooth_order(op, 8);
    const int64_t npts = g->nelem * nqd * nqd;
    DevBuf d_pts, d_gl, d_geo, d_dens;
    std::vector<double> gl = gauss_table();
    if ((st = upload(d_pts, points, size_t(3) * npt, nullptr))) return st;
    if ((st = upload(d_gl, gl.data(), gl.size(), nullptr))) return st;
    if ((st = alloc(d_geo, size_t(npts) * 8 * sizeof(double), nullptr))) return st;
    if ((st = alloc(d_dens, size_t(ndir) * npts * sizeof(double2), nullptr))) return st;
    QuadGeoArgs A{g->d_bez.as<double>(), g->d_pg.as<int>(), g->d_C1.as<double>(), d_gl.as<double>(),
                  g->nel1, g->p, nqd, g->nelem};
    const bool hard = op->bc == IGB_HARD;
    const double2* C = reinterpret_cast<const double2*>(coeffs);
    const igb_op sp = op->sum_parts.empty() ? op : op->sum_parts.front();   // holds the space maps
    const int* s2s0 = hard ? sp->d_s2_to_s0.as<int>() : nullptr;
    if ((st = with_degree(g->p, "potential", [&](auto deg) {
             constexpr int P = decltype(deg)::value;
             hipLaunchKernelGGL(density_points<P>, dim3(unsigned((npts + 255) / 256)), dim3(256), 0, s, A, C,
                                ndir, op->N, s2s0, g->k, d_geo.as<double>(), d_dens.as<double2>());
             return IGB_OK;
         })))
        return st;
    hipLaunchKernelGGL(potential_sum, dim3(unsigned(npt), unsigned(ndir)), dim3(256), 0, s, d_geo.as<double>(),
                       d_dens.as<double2>(), npts, d_pts.as<double>(), npt, op->kappa, hard ? 1 : 0,
                       reinterpret_cast<double2*>(u));
    IGB_HIP(hipGetLastError());
    IGB_HIP(hipStreamSynchronize(s));
    return IGB_OK;
}


igb_status potential_h2_device(igb_op op, const double* coeffs, int ndir, const double* points, int npt, double* u,
                               hipStream_t s) {
    for (int i = 0; i < 3 * npt; ++i)
        if (!std::isfinite(points[i])) {
            set_error("potential_h2: point %d is not finite", i / 3);
            return IGB_ERR_ARG;
        }
    // geometry, q and the transfers of the first part of a separate-form operator
    const igb_op sp = op->sum_parts.empty() ? op : op->sum_parts.front();
    igb_geom g = sp->geom;
    const bool hard = op->bc == IGB_HARD;
    igb_status st;
    PotentialPlan P;
    if ((st = potential_plan(sp, points, npt, P))) return st;
    const int nbox = int(P.box_ptr.size()) - 1;
    if (nbox == 0) return IGB_OK;
    const int q = sp->q, q1 = q + 1, nq = sp->nq, n3 = nq * q1, lmax = P.lmax;
    const double2* C = reinterpret_cast<const double2*>(coeffs);
    // boundary density and geometry at the quadrature points
    const int nqd = smooth_order(op, 8);
    const int64_t nqtot = g->nelem * nqd * nqd;
    DevBuf d_gl, d_geo, d_dens, d_pts, d_perm, d_bptr, d_blo, d_bhi, d_tch, d_fptr, d_fsrc, d_mptr, d_msrc, d_nptr, d_nleaf,
        d_lbox, d_off, d_nodes, d_mom;
    std::vector<double> gl = gauss_table();
    if ((st = upload(d_gl, gl.data(), gl.size(), nullptr))) return st;
    if ((st = alloc(d_geo, size_t(nqtot) * 8 * sizeof(double), nullptr))) return st;
    if ((st = alloc(d_dens, size_t(ndir) * nqtot * sizeof(double2), nullptr))) return st;
    QuadGeoArgs A{g->d_bez.as<double>(), g->d_pg.as<int>(), g->d_C1.as<double>(), d_gl.as<double>(),
                  g->nel1, g->p, nqd, g->nelem};
    const int* s2s0 = hard ? sp->d_s2_to_s0.as<int>() : nullptr;
    if ((st = with_degree(g->p, "potential_h2", [&](auto deg) {
             constexpr int PD = decltype(deg)::value;
             hipLaunchKernelGGL(density_points<PD>, dim3(unsigned((nqtot + 255) / 256)), dim3(256), 0, s, A, C,
                                ndir, op->N, s2s0, g->k, d_geo.as<double>(), d_dens.as<double2>());
             return IGB_OK;
         })))
        return st;
    // source clusters: interpolation nodes, moments of the finest level from the
    // quadrature points, then the coarser levels by the transfers
    std::vector<double> t(q1);
    cheb_nodes(q, t.data());
    const int64_t nclu = P.off[lmax + 1];
    if ((st = upload(d_tch, t.data(), t.size(), nullptr)) || (st = upload(d_off, P.off.data(), P.off.size(), nullptr)) ||
        (st = alloc(d_nodes, size_t(nclu) * nq * 16 * sizeof(double), nullptr)) ||
        (st = alloc(d_mom, size_t(nclu) * nq * ndir * sizeof(double2), nullptr)))
        return st;
    hipLaunchKernelGGL(node_geometry, dim3(unsigned((nclu * nq + 255) / 256)), dim3(256), 0, s, g->d_bez.as<double>(),
                       g->d_pg.as<int>(), g->nel1, g->npatch, lmax, d_off.as<int64_t>(), d_tch.as<double>(), q,
                       d_nodes.as<double>());
    double2* mom = d_mom.as<double2>();
    hipLaunchKernelGGL(pot_leaf_moments, dim3(unsigned(clusters_on_level(g->npatch, lmax)), unsigned(ndir)), dim3(256),
                       0, s, d_geo.as<double>(), d_dens.as<double2>(), nqtot, d_gl.as<double>(), nqd, g->nel1, lmax,
                       1 << (g->m - lmax), d_tch.as<double>(), q, ndir, mom + P.off[lmax] * nq * ndir);
    launch_m2m_levels(sp->d_T.as<double>(), q, lmax, g->npatch, P.off, mom, ndir, s);
    IGB_HIP(hipGetLastError());
    if ((st = upload(d_pts, points, size_t(3) * npt, nullptr)) || (st = upload(d_perm, P.perm.data(), P.perm.size(), nullptr)) ||
        (st = upload(d_bptr, P.box_ptr.data(), P.box_ptr.size(), nullptr)) ||
        (st = upload(d_blo, P.box_lo.data(), P.box_lo.size(), nullptr)) ||
        (st = upload(d_bhi, P.box_hi.data(), P.box_hi.size(), nullptr)) ||
        (st = upload(d_fptr, P.far_ptr.data(), P.far_ptr.size(), nullptr)) ||
        (st = upload(d_nptr, P.near_ptr.data(), P.near_ptr.size(), nullptr)) ||
        (st = upload(d_mptr, P.m2p_ptr.data(), P.m2p_ptr.size(), nullptr)))
        return st;
    if (!P.far_src.empty() && (st = upload(d_fsrc, P.far_src.data(), P.far_src.size(), nullptr))) return st;
    if (!P.m2p_src.empty() && (st = upload(d_msrc, P.m2p_src.data(), P.m2p_src.size(), nullptr))) return st;
    if (!P.near_leaf.empty() && (st = upload(d_nleaf, P.near_leaf.data(), P.near_leaf.size(), nullptr))) return st;
    const bool any_far = !P.far_src.empty();
    if (any_far) {
        if ((st = alloc(d_lbox, size_t(nbox) * n3 * ndir * sizeof(double2), nullptr))) return st;
        hipLaunchKernelGGL(pot_box_m2l, dim3(unsigned(nbox), unsigned(ndir)), dim3(256), 0, s, d_nodes.as<double>(),
                           mom, q, d_blo.as<double>(), d_bhi.as<double>(), d_tch.as<double>(), d_fptr.as<int>(),
                           d_fsrc.as<int>(), ndir, op->kappa, hard ? 1 : 0, d_lbox.as<double2>());
        IGB_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(pot_l2p_near, dim3(unsigned(nbox), unsigned(ndir)), dim3(POT_LEAF_POINTS), 0, s,
                       d_pts.as<double>(), d_perm.as<int>(), d_bptr.as<int>(), d_blo.as<double>(), d_bhi.as<double>(),
                       d_tch.as<double>(), q, any_far ? d_lbox.as<double2>() : nullptr, ndir, d_mptr.as<int>(),
                       d_msrc.as<int>(), d_nodes.as<double>(), mom, d_nptr.as<int>(), d_nleaf.as<int>(),
                       g->m - lmax, lmax, g->nel1, nqd * nqd, d_geo.as<double>(), d_dens.as<double2>(), nqtot,
                       op->kappa, hard ? 1 : 0, npt, reinterpret_cast<double2*>(u));
    IGB_HIP(hipGetLastError());
    IGB_HIP(hipStreamSynchronize(s));   // temporaries are freed on return
    return IGB_OK;
}

}  // namespace igb

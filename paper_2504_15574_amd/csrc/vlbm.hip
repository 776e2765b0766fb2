// vlbm.hip -- HIP (gfx950) implementation of the C ABI in include/vlbm.h.
//
// The vielbein lattice Boltzmann update on the sphere (arXiv:2504.15574,
// Sec. III): per SSP-RK3 stage one fused kernel evaluates the operator L of
// eq. (Lf) -- WENO-5 flux-form advection in theta and phi (Sec. III.E), the
// Hermite-projected inertial force (Sec. III.C), BGK toward the order-3
// equilibrium (Sec. III.B, App. A.2) -- and the Runge-Kutta combination
// (Sec. III.G), with periodic and pole ghosts (Sec. III.F) resolved while the
// tile is staged into LDS.
//
// Populations are stored as deviations g_k = f_k - w_k rho0 (FP64, FP32 or
// scaled FP16).  The rest-state part w_k rho0 of the advection and force is
// exact per theta row, so it is folded into FP64 row tables computed on the
// host; kernels only ever add small quantities.  In exact arithmetic this is
// the same operator as on f itself.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/vlbm.h"

namespace {

constexpr int NQ = 4;    // nodes per axis
constexpr int NK = 16;   // populations
constexpr int NGH = 3;   // ghost layers of the 6-point WENO-5 stencil

// ---------------------------------------------------------------------------
// error reporting
thread_local char g_err[512] = "";

vlbm_status fail(vlbm_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

#define HIP_OK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(VLBM_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// constant tables passed by value to every kernel
struct Consts {
    double v[NQ];         // ascending Gauss-Hermite nodes (roots of H_4)
    double wk[NK];        // product weights w_k
    double K[NQ * NQ];    // K^H,  row k, column k'
    double Kt[NQ * NQ];   // K~^H
    double scale[NK];     // FP16 storage scale 2^e_k (1 for the other formats)
    double iscale[NK];    // 1 / scale
};

// per-row tables in the workspace (FP64)
struct Rows {
    const double* sinv;      // [nt + 6]: sin((j + 1/2) dth), j = -3 .. nt+2 (signed)
    const double* inv_sdth;  // [nt]: 1 / (R sin th_s dth)
    const double* inv_sdph;  // [nt]: 1 / (R sin th_s dph)
    const double* cot;       // [nt]: cos th_s / (R sin th_s)
    const double* rest;      // [16][nt]: L of the rest state w_k rho0
    const double* dC;        // [2][nt + 1][2]: C1 - C2, C3 - C2 of sin th per interface
};

struct StageArgs {
    const void* gin;   // stage input (halo reads)
    const void* gn;    // f_n deviations (point reads), may alias out
    void* out;         // stage output
    Rows rows;
    Consts c;
    int nt, np;
    double dt, inv_tau, rho0, eps;
    double a, b;       // out = a g_n + b (g_in + dt L)
};

// ---------------------------------------------------------------------------
// storage formats
struct StF64 {
    using S = double;
    using T = double;
    __device__ static T ld(const S* p, size_t i, double) { return p[i]; }
    __device__ static void st(S* p, size_t i, T v, double) { p[i] = v; }
};
struct StF32 {
    using S = float;
    using T = float;
    __device__ static T ld(const S* p, size_t i, double) { return p[i]; }
    __device__ static void st(S* p, size_t i, T v, double) { p[i] = v; }
};
struct StF16 {
    using S = _Float16;
    using T = float;
    __device__ static T ld(const S* p, size_t i, double isc) { return (float)p[i] * (float)isc; }
    __device__ static void st(S* p, size_t i, T v, double sc) { p[i] = (_Float16)(v * (float)sc); }
};

// ---------------------------------------------------------------------------
// WENO-5 interface flux for a positive advection velocity (eqs. (fluxes_W5),
// (WENO5_delta), (WENO5_sigma)) from the points s-2..s+2.  h: flux function
// V f at the points, f: the populations of the smoothness indicators (a
// deviation gives the same indicators).  Returns the flux and the normalised
// weights omega_1, omega_3 (omega_2 = 1 - omega_1 - omega_3).
template <class T>
__device__ __forceinline__ T weno5p(T h0, T h1, T h2, T h3, T h4, T f0, T f1, T f2, T f3, T f4,
                                    T eps, T& o1, T& o3) {
    const T c13 = T(1.0 / 3.0), c16 = T(1.0 / 6.0), c56 = T(5.0 / 6.0);
    const T c76 = T(7.0 / 6.0), c116 = T(11.0 / 6.0), c1312 = T(13.0 / 12.0);
    T F1 = c13 * h0 - c76 * h1 + c116 * h2;
    T F2 = -c16 * h1 + c56 * h2 + c13 * h3;
    T F3 = c13 * h2 + c56 * h3 - c16 * h4;
    T a1 = f0 - T(2) * f1 + f2, b1 = f0 - T(4) * f1 + T(3) * f2;
    T a2 = f1 - T(2) * f2 + f3, b2 = f1 - f3;
    T a3 = f2 - T(2) * f3 + f4, b3 = T(3) * f2 - T(4) * f3 + f4;
    T s1 = c1312 * a1 * a1 + T(0.25) * b1 * b1;
    T s2 = c1312 * a2 * a2 + T(0.25) * b2 * b2;
    T s3 = c1312 * a3 * a3 + T(0.25) * b3 * b3;
    T e1 = eps + s1, e2 = eps + s2, e3 = eps + s3;
    T q1 = e1 * e1, q2 = e2 * e2, q3 = e3 * e3;
    // alpha_i = delta_i / q_i normalised with one reciprocal
    T n1 = T(0.1) * (q2 * q3), n2 = T(0.6) * (q1 * q3), n3 = T(0.3) * (q1 * q2);
    T r = T(1) / (n1 + n2 + n3);
    o1 = n1 * r;
    o3 = n3 * r;
    T o2 = n2 * r;
    return o1 * F1 + o2 * F2 + o3 * F3;
}

__device__ __forceinline__ int wrap(int q, int np) {
    int r = q % np;
    return r < 0 ? r + np : r;
}

// ---------------------------------------------------------------------------
// Fused RK stage.  Tile: 4 theta rows x 64 phi columns, one cell per thread
// (wave w owns row s0 + w, lane l column q0 + l).  Populations are processed
// one at a time: the population's tile plus a 3-cell halo is staged in LDS
// (pole rows gathered from column q + np/2 and population 15 - k), both
// interface fluxes of each direction are formed from LDS, and the centre
// values are kept in registers for the cell-local terms at the end.
constexpr int TQ = 64, TS = 4, LR = TS + 2 * NGH, LC = TQ + 2 * NGH, LN = LR * LC;

template <class St>
__global__ __launch_bounds__(256) void stage_kernel(StageArgs A) {
    using T = typename St::T;
    using S = typename St::S;
    __shared__ T tile[2][LR][LC];

    const int nt = A.nt, np = A.np;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int q0 = blockIdx.x * TQ, s0 = blockIdx.y * TS;
    const int s = s0 + wv, q = q0 + lane;
    const bool valid = (s < nt) && (q < np);
    const int sc = s < nt ? s : nt - 1;
    const S* __restrict__ gin = static_cast<const S*>(A.gin);
    const size_t plane = (size_t)nt * np;
    const int half = np > 1 ? np / 2 : 0;

    auto load_tile = [&](int k, int buf) {
        const double isc = A.c.iscale[k];
        for (int idx = threadIdx.x; idx < LN; idx += 256) {
            int r = idx / LC, cc = idx - r * LC;
            int ss = s0 - NGH + r, qq = wrap(q0 - NGH + cc, np);
            int kk = k;
            if (ss < 0) {                 // north pole: row -m <- row m-1, phi + pi, v -> -v
                ss = -1 - ss;
                kk = NK - 1 - k;
                qq = wrap(qq + half, np);
            } else if (ss >= nt) {        // south pole: row nt-1+m <- row nt-m
                ss = 2 * nt - 1 - ss;
                kk = NK - 1 - k;
                qq = wrap(qq + half, np);
            }
            ss = ss < 0 ? 0 : (ss >= nt ? nt - 1 : ss);   // rows never used by a valid cell
            tile[buf][r][cc] = St::ld(gin, (size_t)kk * plane + (size_t)ss * np + qq, isc);
        }
    };

    const T eps = T(A.eps);
    const T rho0 = T(A.rho0);
    const T isdth = T(A.rows.inv_sdth[sc]);
    const T isdph = T(A.rows.inv_sdph[sc]);
    T sn[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) sn[m] = T(A.rows.sinv[sc + m]);   // rows s-3 .. s+3

    T acc[NK], gc[NK];

    load_tile(0, 0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        if (k + 1 < NK) load_tile(k + 1, (k + 1) & 1);
        const int buf = k & 1;
        const int kt = k >> 2, kp = k & 3;
        const T vt = T(A.c.v[kt]), vp = T(A.c.v[kp]);
        // theta direction: column of 7 values, flux function h = v sin(theta_j) g_j
        T g7[7], h7[7], p7[7], hp7[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            g7[m] = tile[buf][wv + m][lane + NGH];
            h7[m] = vt * sn[m] * g7[m];
            p7[m] = tile[buf][wv + NGH][lane + m];
            hp7[m] = vp * p7[m];
        }
        T o1p, o3p, o1m, o3m, Ftp, Ftm, Fpp, Fpm, d1, d2;
        const int dir = kt >= 2 ? 0 : 1;   // v_theta > 0 for kt = 2, 3
        if (dir == 0) {
            Ftp = weno5p(h7[1], h7[2], h7[3], h7[4], h7[5], g7[1], g7[2], g7[3], g7[4], g7[5], eps, o1p, o3p);
            Ftm = weno5p(h7[0], h7[1], h7[2], h7[3], h7[4], g7[0], g7[1], g7[2], g7[3], g7[4], eps, o1m, o3m);
        } else {
            Ftp = weno5p(h7[6], h7[5], h7[4], h7[3], h7[2], g7[6], g7[5], g7[4], g7[3], g7[2], eps, o1p, o3p);
            Ftm = weno5p(h7[5], h7[4], h7[3], h7[2], h7[1], g7[5], g7[4], g7[3], g7[2], g7[1], eps, o1m, o3m);
        }
        // rest-state part of the theta flux beyond its linear-weight value
        {
            const double* dC = A.rows.dC + (size_t)dir * (nt + 1) * 2;
            const T vw = vt * T(A.c.wk[k]) * rho0;
            Ftp += vw * ((o1p - T(0.1)) * T(dC[2 * (sc + 1)]) + (o3p - T(0.3)) * T(dC[2 * (sc + 1) + 1]));
            Ftm += vw * ((o1m - T(0.1)) * T(dC[2 * sc]) + (o3m - T(0.3)) * T(dC[2 * sc + 1]));
        }
        if (kp >= 2) {
            Fpp = weno5p(hp7[1], hp7[2], hp7[3], hp7[4], hp7[5], p7[1], p7[2], p7[3], p7[4], p7[5], eps, d1, d2);
            Fpm = weno5p(hp7[0], hp7[1], hp7[2], hp7[3], hp7[4], p7[0], p7[1], p7[2], p7[3], p7[4], eps, d1, d2);
        } else {
            Fpp = weno5p(hp7[6], hp7[5], hp7[4], hp7[3], hp7[2], p7[6], p7[5], p7[4], p7[3], p7[2], eps, d1, d2);
            Fpm = weno5p(hp7[5], hp7[4], hp7[3], hp7[2], hp7[1], p7[5], p7[4], p7[3], p7[2], p7[1], eps, d1, d2);
        }
        acc[k] = T(A.rows.rest[(size_t)k * nt + sc]) - isdth * (Ftp - Ftm) - isdph * (Fpp - Fpm);
        gc[k] = g7[3];
        // keep this population's arithmetic ahead of the barrier: sinking it past
        // the barriers would keep every population's stencil live at once
        asm volatile("" ::"v"(acc[k]));
        __syncthreads();
    }

    if (!valid) return;

    // cell-local terms on the deviations: inertial force (eqs. (df), (Lf)) and BGK
    const T cot = T(A.rows.cot[sc]);
    T v[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) v[i] = T(A.c.v[i]);
    T drho = 0, jt = 0, jp = 0;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        drho += gc[k];
        jt += v[k >> 2] * gc[k];
        jp += v[k & 3] * gc[k];
    }
    const T rho = rho0 + drho;
    const T irho = T(1) / rho;
    const T ut = jt * irho, up = jp * irho;
    const T u2 = ut * ut + up * up;
    const T itau = T(A.inv_tau), dt = T(A.dt);
    const T ca = T(A.a), cb = T(A.b);
    const S* __restrict__ gnp = static_cast<const S*>(A.gn);
    S* outp = static_cast<S*>(A.out);
    const size_t cell = (size_t)s * np + q;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int kt = k >> 2, kp = k & 3;
        T dfdvt = 0, dfvdvp = 0;
#pragma unroll
        for (int b = 0; b < NQ; ++b) {
            dfdvt += T(A.c.K[kt * NQ + b]) * gc[b * NQ + kp];
            dfvdvp += T(A.c.Kt[kp * NQ + b]) * gc[kt * NQ + b];
        }
        const T G = -cot * (v[kp] * v[kp] * dfdvt - v[kt] * dfvdvp);
        const T xi = v[kt] * ut + v[kp] * up;
        const T pm1 = xi + T(0.5) * (xi * xi - u2) + xi * (xi * xi - T(3) * u2) * T(1.0 / 6.0);
        const T C = (T(A.c.wk[k]) * (drho + rho * pm1) - gc[k]) * itau;
        const T L = acc[k] + G + C;
        const T y = gc[k] + dt * L;
        T o = cb * y;
        if (ca != T(0)) o += ca * St::ld(gnp, (size_t)k * plane + cell, A.c.iscale[k]);
        St::st(outp, (size_t)k * plane + cell, o, A.c.scale[k]);
    }
}

// ---------------------------------------------------------------------------
// Equilibrium initialisation: g_k = f^eq_k(rho, u, T) - w_k rho0 with the
// thermal order-2/3 Hermite terms for T != 1, computed in FP64.
template <class St>
__global__ void init_kernel(const double* rho, const double* ut, const double* up,
                            const double* Tf, void* outv, Consts c, int n, double rho0) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    typename St::S* out = static_cast<typename St::S*>(outv);
    const double r = rho[i], a = ut[i], b = up[i];
    const double dT = Tf ? Tf[i] - 1.0 : 0.0;
    const double u2 = a * a + b * b;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const double vt = c.v[k >> 2], vp = c.v[k & 3];
        const double xi = vt * a + vp * b, v2 = vt * vt + vp * vp;
        const double pm1 = xi + 0.5 * (xi * xi - u2 + dT * (v2 - 2.0)) +
                           xi * (xi * xi - 3.0 * u2 + 3.0 * dT * (v2 - 4.0)) / 6.0;
        const double g = c.wk[k] * ((r - rho0) + r * pm1);
        St::st(out, (size_t)k * n + i, (typename St::T)g, c.scale[k]);
    }
}

// f (FP64) <-> stored deviations, populations k0 .. k0+nk-1; f is [nk][n]
template <class St>
__global__ void decode_kernel(const void* inv, double* f, Consts c, int n, double rho0, int k0, int nk) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const typename St::S* in = static_cast<const typename St::S*>(inv);
    for (int j = 0; j < nk; ++j) {
        const int k = k0 + j;
        f[(size_t)j * n + i] = c.wk[k] * rho0 + (double)St::ld(in, (size_t)k * n + i, c.iscale[k]);
    }
}

template <class St>
__global__ void encode_kernel(const double* f, void* outv, Consts c, int n, double rho0, int k0, int nk) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    typename St::S* out = static_cast<typename St::S*>(outv);
    for (int j = 0; j < nk; ++j) {
        const int k = k0 + j;
        St::st(out, (size_t)k * n + i, (typename St::T)(f[(size_t)j * n + i] - c.wk[k] * rho0), c.scale[k]);
    }
}

// Moments in FP64 from the stored deviations (eq. (f_moments_sum)).
template <class St>
__device__ __forceinline__ void cell_moments(const typename St::S* in, size_t i, size_t n,
                                             const Consts& c, double rho0, double& rho,
                                             double& ut, double& up, double& T, double& e,
                                             int& nbad) {
    double g[NK];
    double dr = 0, jt = 0, jp = 0;
    nbad = 0;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        g[k] = (double)St::ld(in, (size_t)k * n + i, c.iscale[k]);
        nbad += isfinite(g[k]) ? 0 : 1;
        dr += g[k];
        jt += c.v[k >> 2] * g[k];
        jp += c.v[k & 3] * g[k];
    }
    rho = rho0 + dr;
    ut = jt / rho;
    up = jp / rho;
    double th = 0, en = 0;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const double f = c.wk[k] * rho0 + g[k];
        const double dt_ = c.v[k >> 2] - ut, dp_ = c.v[k & 3] - up;
        th += f * (dt_ * dt_ + dp_ * dp_);
        en += 0.5 * f * (c.v[k >> 2] * c.v[k >> 2] + c.v[k & 3] * c.v[k & 3]);
    }
    T = th / (2.0 * rho);
    e = en;
}

template <class St>
__global__ void moments_kernel(const void* inv, double* rho, double* ut, double* up, double* T,
                               Consts c, int n, double rho0) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r, a, b, t, e;
    int nb;
    cell_moments<St>(static_cast<const typename St::S*>(inv), i, n, c, rho0, r, a, b, t, e, nb);
    rho[i] = r;
    ut[i] = a;
    up[i] = b;
    if (T) T[i] = t;
}

// Diagnostics: per-block FP64 partial sums, then one block folds the partials
// in a fixed order (deterministic for a given grid).
constexpr int RED_T = 256;

template <class St>
__global__ __launch_bounds__(RED_T) void reduce_kernel(const void* inv, const double* sinv,
                                                       double* part, Consts c, int nt, int np,
                                                       double rho0, double R) {
    __shared__ double sh[8][RED_T];
    const size_t n = (size_t)nt * np;
    const double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    double acc[8] = {0, 0, 0, 0, 0, 0, INFINITY, -INFINITY};
    for (size_t i = (size_t)blockIdx.x * RED_T + threadIdx.x; i < n; i += (size_t)gridDim.x * RED_T) {
        const int s = (int)(i / np);
        const double st = sinv[s + NGH];
        const double dA = R * R * st * dth * dph;
        double r, a, b, t, e;
        int nb;
        cell_moments<St>(static_cast<const typename St::S*>(inv), i, n, c, rho0, r, a, b, t, e, nb);
        acc[0] += dA * r;
        acc[1] += dA * e;
        acc[2] += dA * 0.5 * r * (a * a + b * b);
        acc[3] += dA * r * b * R * st;
        acc[4] += nb;
        const double u = sqrt(a * a + b * b);
        acc[5] = fmax(acc[5], u);
        acc[6] = fmin(acc[6], r);
        acc[7] = fmax(acc[7], r);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) sh[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int w = RED_T / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int j = 0; j < 5; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + w];
            sh[5][threadIdx.x] = fmax(sh[5][threadIdx.x], sh[5][threadIdx.x + w]);
            sh[6][threadIdx.x] = fmin(sh[6][threadIdx.x], sh[6][threadIdx.x + w]);
            sh[7][threadIdx.x] = fmax(sh[7][threadIdx.x], sh[7][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) part[(size_t)blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void reduce_final(const double* part, int nblk, double* out) {
    if (threadIdx.x != 0) return;
    double acc[8] = {0, 0, 0, 0, 0, 0, INFINITY, -INFINITY};
    for (int b = 0; b < nblk; ++b) {
        for (int j = 0; j < 5; ++j) acc[j] += part[(size_t)b * 8 + j];
        acc[5] = fmax(acc[5], part[(size_t)b * 8 + 5]);
        acc[6] = fmin(acc[6], part[(size_t)b * 8 + 6]);
        acc[7] = fmax(acc[7], part[(size_t)b * 8 + 7]);
    }
    for (int j = 0; j < 8; ++j) out[j] = acc[j];
}

// Vorticity from the FP64 velocity fields, fourth-order central differences.
// Across a pole both the velocity (v -> -v at phi + pi) and sin th change sign,
// so u_phi sin th continues evenly to column q + np/2.
__global__ void vorticity_kernel(const double* ut, const double* up, const double* sinv,
                                 double* om, int nt, int np, double R) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x, s = blockIdx.y;
    if (q >= np || s >= nt) return;
    const double dth = M_PI / nt, dph = 2.0 * M_PI / np;
    const int half = np > 1 ? np / 2 : 0;
    double g[5];
#pragma unroll
    for (int m = -2; m <= 2; ++m) {
        int j = s + m, qq = q;
        if (j < 0 || j >= nt) {
            qq = (q + half) % np;
            j = j < 0 ? -1 - j : 2 * nt - 1 - j;
        }
        g[m + 2] = up[(size_t)j * np + qq] * sinv[j + NGH];
    }
    const double dg = (g[0] - 8.0 * g[1] + 8.0 * g[3] - g[4]) / (12.0 * dth);
    double du = 0.0;
    if (np > 1) {
        double u[5];
#pragma unroll
        for (int m = -2; m <= 2; ++m) u[m + 2] = ut[(size_t)s * np + wrap(q + m, np)];
        du = (u[0] - 8.0 * u[1] + 8.0 * u[3] - u[4]) / (12.0 * dph);
    }
    om[(size_t)s * np + q] = (dg - du) / (R * sinv[s + NGH]);
}

// ---------------------------------------------------------------------------
// host-side tables (FP64), written from Sec. III.A / III.C / App. A.2
double hermite(int n, double x) {
    if (n < 0) return 0.0;
    double a = 1.0, b = x;   // H_0, H_1
    if (n == 0) return a;
    for (int m = 1; m < n; ++m) {
        double c = x * b - m * a;
        a = b;
        b = c;
    }
    return b;
}

void build_consts(Consts& c, int storage) {
    const double r6 = std::sqrt(6.0);
    c.v[0] = -std::sqrt(3.0 + r6);
    c.v[1] = -std::sqrt(3.0 - r6);
    c.v[2] = std::sqrt(3.0 - r6);
    c.v[3] = std::sqrt(3.0 + r6);
    double w1[NQ];
    for (int i = 0; i < NQ; ++i) {
        const double h5 = hermite(5, c.v[i]);
        w1[i] = 24.0 / (h5 * h5);          // Q! / H_{Q+1}(v)^2 with Q = 4
    }
    for (int k = 0; k < NK; ++k) c.wk[k] = w1[k >> 2] * w1[k & 3];
    const double fact[NQ] = {1.0, 1.0, 2.0, 6.0};
    for (int i = 0; i < NQ; ++i)
        for (int j = 0; j < NQ; ++j) {
            double a = 0.0, b = 0.0;
            for (int l = 0; l < NQ; ++l) {
                const double hl1 = hermite(l + 1, c.v[i]) / fact[l];
                a += hl1 * hermite(l, c.v[j]);
                b += hl1 * (hermite(l + 1, c.v[j]) + l * hermite(l - 1, c.v[j]));
            }
            c.K[i * NQ + j] = -w1[i] * a;
            c.Kt[i * NQ + j] = -w1[i] * b;
        }
    for (int k = 0; k < NK; ++k) {
        double sc = 1.0;
        if (storage == VLBM_STORE_F16_DEV) sc = std::ldexp(1.0, 10 - (int)std::lround(std::log2(c.wk[k])));
        c.scale[k] = sc;
        c.iscale[k] = 1.0 / sc;
    }
}

// Rest-state tables for a grid.  With g = 0 the populations are w_k rho0; the
// theta flux then has smoothness indicators sigma = 0 only where the data are
// uniform, so the kernel adds the nonlinear-weight part from dC at run time and
// the linear-weight part is folded into rest[] together with the force on w rho0.
struct HostRows {
    std::vector<double> sinv, inv_sdth, inv_sdph, cot, rest, dC;
};

void build_rows(HostRows& h, const vlbm_params& p, const Consts& c) {
    const int nt = p.n_theta, np = p.n_phi;
    const double dth = M_PI / nt, dph = 2.0 * M_PI / np, R = p.radius;
    h.sinv.resize(nt + 2 * NGH);
    for (int j = -NGH; j < nt + NGH; ++j) h.sinv[j + NGH] = std::sin((j + 0.5) * dth);
    h.inv_sdth.resize(nt);
    h.inv_sdph.resize(nt);
    h.cot.resize(nt);
    for (int s = 0; s < nt; ++s) {
        const double th = (s + 0.5) * dth;
        h.inv_sdth[s] = 1.0 / (R * std::sin(th) * dth);
        h.inv_sdph[s] = 1.0 / (R * std::sin(th) * dph);
        h.cot[s] = std::cos(th) / (R * std::sin(th));
    }
    // candidate reconstructions of S_j = sin th_j at interface i (= s + 1/2, s = i - 1)
    h.dC.assign(2 * (nt + 1) * 2, 0.0);
    std::vector<double> clin(2 * (nt + 1));
    for (int dir = 0; dir < 2; ++dir)
        for (int i = 0; i <= nt; ++i) {
            const int s = i - 1;
            double P[5];
            for (int m = 0; m < 5; ++m) {
                const int j = dir == 0 ? s - 2 + m : s + 3 - m;   // mirrored stencil
                P[m] = h.sinv[j + NGH];
            }
            const double C1 = P[0] / 3.0 - 7.0 * P[1] / 6.0 + 11.0 * P[2] / 6.0;
            const double C2 = -P[1] / 6.0 + 5.0 * P[2] / 6.0 + P[3] / 3.0;
            const double C3 = P[2] / 3.0 + 5.0 * P[3] / 6.0 - P[4] / 6.0;
            h.dC[(dir * (nt + 1) + i) * 2 + 0] = C1 - C2;
            h.dC[(dir * (nt + 1) + i) * 2 + 1] = C3 - C2;
            clin[dir * (nt + 1) + i] = 0.1 * C1 + 0.6 * C2 + 0.3 * C3;
        }
    h.rest.assign((size_t)NK * nt, 0.0);
    const double r0 = p.rho0;
    for (int k = 0; k < NK; ++k) {
        const int kt = k >> 2, kp = k & 3;
        const int dir = c.v[kt] > 0 ? 0 : 1;
        for (int s = 0; s < nt; ++s) {
            const double vw = c.v[kt] * c.wk[k] * r0;
            const double adv = -h.inv_sdth[s] * vw * (clin[dir * (nt + 1) + s + 1] - clin[dir * (nt + 1) + s]);
            double dfdvt = 0.0, dfvdvp = 0.0;
            for (int b = 0; b < NQ; ++b) {
                dfdvt += c.K[kt * NQ + b] * c.wk[b * NQ + kp] * r0;
                dfvdvp += c.Kt[kp * NQ + b] * c.wk[kt * NQ + b] * r0;
            }
            const double G = -h.cot[s] * (c.v[kp] * c.v[kp] * dfdvt - c.v[kt] * dfvdvp);
            h.rest[(size_t)k * nt + s] = adv + G;
        }
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

size_t store_bytes(int storage) {
    return storage == VLBM_STORE_F64 ? 8 : storage == VLBM_STORE_F32_DEV ? 4 : 2;
}

constexpr int RED_BLOCKS = 1024;

struct Layout {
    size_t fbuf[3], sinv, inv_sdth, inv_sdph, cot, rest, dC, fields, part, dout, total;
};

Layout layout_of(const vlbm_params& p) {
    Layout L{};
    const size_t n = (size_t)p.n_theta * p.n_phi;
    size_t off = 0;
    const size_t fb = align_up(NK * n * store_bytes(p.storage));
    for (int i = 0; i < 3; ++i) { L.fbuf[i] = off; off += fb; }
    L.sinv = off; off += align_up(sizeof(double) * (p.n_theta + 2 * NGH));
    L.inv_sdth = off; off += align_up(sizeof(double) * p.n_theta);
    L.inv_sdph = off; off += align_up(sizeof(double) * p.n_theta);
    L.cot = off; off += align_up(sizeof(double) * p.n_theta);
    L.rest = off; off += align_up(sizeof(double) * NK * p.n_theta);
    L.dC = off; off += align_up(sizeof(double) * 4 * (p.n_theta + 1));
    L.fields = off; off += align_up(sizeof(double) * 4 * n);
    L.part = off; off += align_up(sizeof(double) * 8 * RED_BLOCKS);
    L.dout = off; off += align_up(sizeof(double) * 8);
    L.total = off;
    return L;
}

vlbm_status check_params(const vlbm_params* p) {
    if (!p) return fail(VLBM_ERR_ARG, "params is NULL");
    if (p->abi_version != VLBM_ABI_VERSION)
        return fail(VLBM_ERR_ARG, "abi_version %u != %u", p->abi_version, VLBM_ABI_VERSION);
    if (p->n_theta < NGH) return fail(VLBM_ERR_ARG, "n_theta must be >= 3");
    if (p->n_phi < 1 || (p->n_phi > 1 && (p->n_phi & 1)))
        return fail(VLBM_ERR_ARG, "n_phi must be 1 or even");
    if ((long long)p->n_theta * p->n_phi > (1LL << 31) - 1)
        return fail(VLBM_ERR_ARG, "grid too large");
    if (!(p->radius > 0) || !(p->tau > 0) || !(p->dt > 0) || !(p->rho0 > 0) || !(p->weno_eps > 0))
        return fail(VLBM_ERR_ARG, "radius, tau, dt, rho0 and weno_eps must be > 0");
    if (!std::isfinite(p->radius) || !std::isfinite(p->tau) || !std::isfinite(p->dt) ||
        !std::isfinite(p->rho0) || !std::isfinite(p->weno_eps))
        return fail(VLBM_ERR_ARG, "non-finite parameter");
    if (p->q != 4) return fail(VLBM_ERR_UNSUPPORTED, "only q = 4 (D2Q16) is implemented");
    if (p->storage < 0 || p->storage > 2) return fail(VLBM_ERR_UNSUPPORTED, "unknown storage %d", p->storage);
    if (p->advection != VLBM_ADV_WENO5) return fail(VLBM_ERR_UNSUPPORTED, "unknown advection %d", p->advection);
    return VLBM_OK;
}

}  // namespace

struct vlbm_ctx {
    vlbm_params p;
    hipStream_t stream;
    char* ws;
    Layout L;
    Consts c;
    int64_t launches;
    int device;
};

namespace {

template <class T>
T* at(vlbm_ctx* x, size_t off) { return reinterpret_cast<T*>(x->ws + off); }

int n_cells(const vlbm_ctx* x) { return x->p.n_theta * x->p.n_phi; }

vlbm_status launch_check() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VLBM_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return VLBM_OK;
}

template <class St>
vlbm_status launch_stage(vlbm_ctx* x, int stage) {
    StageArgs A;
    const int nt = x->p.n_theta, np = x->p.n_phi;
    void* fn = x->ws + x->L.fbuf[0];
    void* fa = x->ws + x->L.fbuf[1];
    void* fb = x->ws + x->L.fbuf[2];
    A.rows.sinv = at<double>(x, x->L.sinv);
    A.rows.inv_sdth = at<double>(x, x->L.inv_sdth);
    A.rows.inv_sdph = at<double>(x, x->L.inv_sdph);
    A.rows.cot = at<double>(x, x->L.cot);
    A.rows.rest = at<double>(x, x->L.rest);
    A.rows.dC = at<double>(x, x->L.dC);
    A.c = x->c;
    A.nt = nt;
    A.np = np;
    A.dt = x->p.dt;
    A.inv_tau = 1.0 / x->p.tau;
    A.rho0 = x->p.rho0;
    A.eps = x->p.weno_eps;
    A.gn = fn;
    if (stage == 1) { A.gin = fn; A.out = fa; A.a = 0.0; A.b = 1.0; }
    else if (stage == 2) { A.gin = fa; A.out = fb; A.a = 0.75; A.b = 0.25; }
    else { A.gin = fb; A.out = fn; A.a = 1.0 / 3.0; A.b = 2.0 / 3.0; }
    dim3 grid((np + TQ - 1) / TQ, (nt + TS - 1) / TS);
    hipLaunchKernelGGL(stage_kernel<St>, grid, dim3(256), 0, x->stream, A);
    x->launches++;
    return launch_check();
}

template <class F>
vlbm_status dispatch(int storage, F&& f) {
    switch (storage) {
        case VLBM_STORE_F64: return f(StF64{});
        case VLBM_STORE_F32_DEV: return f(StF32{});
        default: return f(StF16{});
    }
}

vlbm_status copy_in(vlbm_ctx* x, double* dst, const double* src, size_t n, int on_dev) {
    HIP_OK(hipMemcpyAsync(dst, src, n * sizeof(double),
                          on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, x->stream));
    return VLBM_OK;
}

}  // namespace

extern "C" {

size_t vlbm_workspace_bytes(const vlbm_params* p) {
    if (check_params(p) != VLBM_OK) return 0;
    return layout_of(*p).total;
}

double vlbm_suggest_dt(const vlbm_params* p) {
    if (!p || p->n_theta < 1 || p->n_phi < 1 || !(p->tau > 0) || !(p->radius > 0)) return 0.0;
    const double dth = M_PI / p->n_theta;
    double dt = std::fmin(0.2 * dth, p->tau);
    if (p->n_phi > 1) {
        const double dph = 2.0 * M_PI / p->n_phi;
        const double vmax = std::sqrt(3.0 + std::sqrt(6.0));
        dt = std::fmin(dt, 0.5 * p->radius * std::sin(0.5 * dth) * dph / vmax);
    }
    return dt;
}

vlbm_status vlbm_create(const vlbm_params* p, void* hip_stream, void* workspace,
                        size_t workspace_bytes, vlbm_ctx** out) {
    g_err[0] = 0;
    vlbm_status st = check_params(p);
    if (st != VLBM_OK) return st;
    if (!out || !workspace) return fail(VLBM_ERR_ARG, "out and workspace must not be NULL");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(VLBM_ERR_ARG, "workspace must be 256-byte aligned");
    const Layout L = layout_of(*p);
    if (workspace_bytes < L.total)
        return fail(VLBM_ERR_ALLOC, "workspace of %zu bytes < required %zu", workspace_bytes, L.total);
    vlbm_ctx* x = new (std::nothrow) vlbm_ctx();
    if (!x) return fail(VLBM_ERR_ALLOC, "host allocation failed");
    x->p = *p;
    x->stream = static_cast<hipStream_t>(hip_stream);
    x->ws = static_cast<char*>(workspace);
    x->L = L;
    x->launches = 0;
    build_consts(x->c, p->storage);
    HostRows h;
    build_rows(h, *p, x->c);
    hipError_t e = hipGetDevice(&x->device);
    const struct { size_t off; const std::vector<double>* v; } up[] = {
        {L.sinv, &h.sinv}, {L.inv_sdth, &h.inv_sdth}, {L.inv_sdph, &h.inv_sdph},
        {L.cot, &h.cot}, {L.rest, &h.rest}, {L.dC, &h.dC}};
    for (const auto& u : up) {
        if (e != hipSuccess) break;
        e = hipMemcpyAsync(x->ws + u.off, u.v->data(), u.v->size() * sizeof(double),
                           hipMemcpyHostToDevice, x->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
    if (e != hipSuccess) {
        delete x;
        return fail(VLBM_ERR_DEVICE, "table upload failed: %s", hipGetErrorString(e));
    }
    *out = x;
    return VLBM_OK;
}

vlbm_status vlbm_destroy(vlbm_ctx* x) {
    delete x;
    return VLBM_OK;
}

vlbm_status vlbm_init_fields(vlbm_ctx* x, const double* rho, const double* ut, const double* up,
                             const double* T, int on_dev) {
    if (!x || !rho || !ut || !up) return fail(VLBM_ERR_ARG, "NULL argument");
    const int n = n_cells(x);
    double* F = at<double>(x, x->L.fields);
    vlbm_status st;
    if ((st = copy_in(x, F, rho, n, on_dev))) return st;
    if ((st = copy_in(x, F + n, ut, n, on_dev))) return st;
    if ((st = copy_in(x, F + 2 * (size_t)n, up, n, on_dev))) return st;
    const double* Tp = nullptr;
    if (T) {
        if ((st = copy_in(x, F + 3 * (size_t)n, T, n, on_dev))) return st;
        Tp = F + 3 * (size_t)n;
    }
    void* fn = x->ws + x->L.fbuf[0];
    st = dispatch(x->p.storage, [&](auto tag) {
        using St = decltype(tag);
        hipLaunchKernelGGL(init_kernel<St>, dim3((n + 255) / 256), dim3(256), 0, x->stream,
                           F, F + n, F + 2 * (size_t)n, Tp, fn, x->c, n, x->p.rho0);
        return launch_check();
    });
    if (st) return st;
    if (!on_dev) HIP_OK(hipStreamSynchronize(x->stream));
    return VLBM_OK;
}

vlbm_status vlbm_step(vlbm_ctx* x, int64_t n_steps) {
    if (!x || n_steps < 0) return fail(VLBM_ERR_ARG, "bad context or n_steps < 0");
    for (int64_t i = 0; i < n_steps; ++i)
        for (int stage = 1; stage <= 3; ++stage) {
            vlbm_status st = dispatch(x->p.storage, [&](auto tag) {
                return launch_stage<decltype(tag)>(x, stage);
            });
            if (st) return st;
        }
    return VLBM_OK;
}

vlbm_status vlbm_moments(vlbm_ctx* x, double* rho, double* ut, double* up, double* T, int on_dev) {
    if (!x || !rho || !ut || !up) return fail(VLBM_ERR_ARG, "NULL argument");
    const int n = n_cells(x);
    double* F = at<double>(x, x->L.fields);
    double *dr = rho, *da = ut, *db = up, *dT = T;
    if (!on_dev) { dr = F; da = F + n; db = F + 2 * (size_t)n; dT = T ? F + 3 * (size_t)n : nullptr; }
    const void* fn = x->ws + x->L.fbuf[0];
    vlbm_status st = dispatch(x->p.storage, [&](auto tag) {
        using St = decltype(tag);
        hipLaunchKernelGGL(moments_kernel<St>, dim3((n + 255) / 256), dim3(256), 0, x->stream,
                           fn, dr, da, db, dT, x->c, n, x->p.rho0);
        return launch_check();
    });
    if (st) return st;
    if (!on_dev) {
        HIP_OK(hipMemcpyAsync(rho, dr, n * sizeof(double), hipMemcpyDeviceToHost, x->stream));
        HIP_OK(hipMemcpyAsync(ut, da, n * sizeof(double), hipMemcpyDeviceToHost, x->stream));
        HIP_OK(hipMemcpyAsync(up, db, n * sizeof(double), hipMemcpyDeviceToHost, x->stream));
        if (T) HIP_OK(hipMemcpyAsync(T, dT, n * sizeof(double), hipMemcpyDeviceToHost, x->stream));
        HIP_OK(hipStreamSynchronize(x->stream));
    }
    return VLBM_OK;
}

vlbm_status vlbm_vorticity(vlbm_ctx* x, double* om, int on_dev) {
    if (!x || !om) return fail(VLBM_ERR_ARG, "NULL argument");
    const int n = n_cells(x);
    double* F = at<double>(x, x->L.fields);
    vlbm_status st = vlbm_moments(x, F, F + n, F + 2 * (size_t)n, nullptr, 1);
    if (st) return st;
    double* dst = on_dev ? om : F + 3 * (size_t)n;
    dim3 grid((x->p.n_phi + 127) / 128, x->p.n_theta);
    hipLaunchKernelGGL(vorticity_kernel, grid, dim3(128), 0, x->stream, F + n, F + 2 * (size_t)n,
                       at<double>(x, x->L.sinv), dst, x->p.n_theta, x->p.n_phi, x->p.radius);
    if ((st = launch_check())) return st;
    if (!on_dev) {
        HIP_OK(hipMemcpyAsync(om, dst, n * sizeof(double), hipMemcpyDeviceToHost, x->stream));
        HIP_OK(hipStreamSynchronize(x->stream));
    }
    return VLBM_OK;
}

vlbm_status vlbm_diagnostics(vlbm_ctx* x, double out[8]) {
    if (!x || !out) return fail(VLBM_ERR_ARG, "NULL argument");
    const int n = n_cells(x);
    int nblk = (n + RED_T - 1) / RED_T;
    if (nblk > RED_BLOCKS) nblk = RED_BLOCKS;
    double* part = at<double>(x, x->L.part);
    double* dout = at<double>(x, x->L.dout);
    const void* fn = x->ws + x->L.fbuf[0];
    vlbm_status st = dispatch(x->p.storage, [&](auto tag) {
        using St = decltype(tag);
        hipLaunchKernelGGL(reduce_kernel<St>, dim3(nblk), dim3(RED_T), 0, x->stream, fn,
                           at<double>(x, x->L.sinv), part, x->c, x->p.n_theta, x->p.n_phi,
                           x->p.rho0, x->p.radius);
        return launch_check();
    });
    if (st) return st;
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(64), 0, x->stream, part, nblk, dout);
    if ((st = launch_check())) return st;
    HIP_OK(hipMemcpyAsync(out, dout, 8 * sizeof(double), hipMemcpyDeviceToHost, x->stream));
    HIP_OK(hipStreamSynchronize(x->stream));
    if (out[4] > 0) return fail(VLBM_ERR_UNSTABLE, "%.0f non-finite populations", out[4]);
    return VLBM_OK;
}

// Host transfers go through the FP64 field staging area (4 planes) in chunks
// of four populations, so no device memory is allocated here.
vlbm_status vlbm_get_populations(vlbm_ctx* x, double* f, int on_dev) {
    if (!x || !f) return fail(VLBM_ERR_ARG, "NULL argument");
    const int n = n_cells(x);
    const void* fn = x->ws + x->L.fbuf[0];
    double* F = at<double>(x, x->L.fields);
    for (int k0 = 0; k0 < NK; k0 += 4) {
        double* dst = on_dev ? f + (size_t)k0 * n : F;
        vlbm_status st = dispatch(x->p.storage, [&](auto tag) {
            using St = decltype(tag);
            hipLaunchKernelGGL(decode_kernel<St>, dim3((n + 255) / 256), dim3(256), 0, x->stream, fn,
                               dst, x->c, n, x->p.rho0, k0, 4);
            return launch_check();
        });
        if (st) return st;
        if (!on_dev) {
            HIP_OK(hipMemcpyAsync(f + (size_t)k0 * n, F, 4 * (size_t)n * sizeof(double),
                                  hipMemcpyDeviceToHost, x->stream));
            HIP_OK(hipStreamSynchronize(x->stream));
        }
    }
    return VLBM_OK;
}

vlbm_status vlbm_set_populations(vlbm_ctx* x, const double* f, int on_dev) {
    if (!x || !f) return fail(VLBM_ERR_ARG, "NULL argument");
    const int n = n_cells(x);
    void* fn = x->ws + x->L.fbuf[0];
    double* F = at<double>(x, x->L.fields);
    for (int k0 = 0; k0 < NK; k0 += 4) {
        const double* src = on_dev ? f + (size_t)k0 * n : F;
        if (!on_dev)
            HIP_OK(hipMemcpyAsync(F, f + (size_t)k0 * n, 4 * (size_t)n * sizeof(double),
                                  hipMemcpyHostToDevice, x->stream));
        vlbm_status st = dispatch(x->p.storage, [&](auto tag) {
            using St = decltype(tag);
            hipLaunchKernelGGL(encode_kernel<St>, dim3((n + 255) / 256), dim3(256), 0, x->stream, src,
                               fn, x->c, n, x->p.rho0, k0, 4);
            return launch_check();
        });
        if (st) return st;
        if (!on_dev) HIP_OK(hipStreamSynchronize(x->stream));
    }
    return VLBM_OK;
}

int64_t vlbm_stage_launches(const vlbm_ctx* x) { return x ? x->launches : -1; }

const char* vlbm_last_error(void) { return g_err; }

}  // extern "C"

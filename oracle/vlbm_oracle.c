/*
 * vlbm_oracle.c -- plain, slow, FP64 CPU reference of the vielbein lattice
 * Boltzmann method (vLBM) on the sphere, arXiv:2504.15574 (Ambrus, Bellantoni,
 * Busuioc, Gabbana, Toschi).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline of the benchmark are the only code that may load this library.
 * It shares no code, header, table or helper with the HIP library; it is
 * written from the paper alone, in the paper's order and notation:
 *
 *   Sec. III.A  velocity set: Gauss-Hermite nodes (roots of H_Q) and weights,
 *               eq. (GH_weights); product rules D2Q9 (Q = 3, App. A.1) and
 *               D2Q16 (Q = 4, App. A.2 Table IV).
 *   Sec. III.B  BGK collision; truncated equilibrium, eqs. (feq_Q=3),
 *               (feq_Q=4).
 *   Sec. III.C  velocity derivatives by the kernels K^H, K~^H, eqs. (df),
 *               (kernels).
 *   Sec. III.D  cell-centred grid, eq. (discrete_coord_sphere).
 *   Sec. III.E  flux-form advection, eq. (discrete_advection_sphere); WENO-5
 *               fluxes, eqs. (fluxes_W5), (WENO5_delta), (WENO5_sigma); the
 *               upwind fluxes U1, U2, U3, eq. (fluxes_U1-3); the "Komissarov"
 *               form of the theta derivative, eqs. (Komissarov_scheme),
 *               (Komissarov_sin_cos).
 *   Sec. III.F  periodic phi ghosts, eq. (bcs_phi); pole ghosts, eq.
 *               (bcs_theta).
 *   Sec. III.G  SSP-RK3 and the operator L[f], eq. (Lf).
 *
 * Readings taken where the paper is silent or ambiguous:
 *   - theta flux: the WENO candidates reconstruct the flux function
 *     h_j = v_k sin(theta_j) f_j point by point (V taken at each stencil
 *     point); the smoothness indicators use f as printed in eq. (WENO5_sigma);
 *   - the nonlinear weights are delta_j/(eps + sigma_j)^2 (the printed form has
 *     no eps and divides by zero on smooth data);
 *   - the upwind side is the sign of v_k (the node component), for the pole
 *     interfaces too, where sin(theta) = 0; the other side uses the mirrored
 *     stencil (index s+m replaced by s+1-m);
 *   - across a pole the whole velocity is inverted (population k -> 15-k for
 *     ascending nodes) and ghost rows keep the signed sin(theta) of their
 *     (negative or > pi) polar angle;
 *   - the collision is isothermal with T0 = 1; an initial temperature T != 1
 *     only enters the initial populations through the order-3 Hermite
 *     projection of a Maxwellian at temperature T.
 *
 * Indexing: populations k = Q*kt + kp, kt (theta component) and kp (phi
 * component) index the ascending nodes v_0 < ... < v_{Q-1}.  Fields are
 * [Q^2][n_theta][n_phi] (phi fastest), 0-based s with theta_s = (s+1/2)pi/Nt
 * and phi_q = (q+1/2)2pi/Np.  The quadrature order Q (3 or 4, default 4) is
 * a process-wide model choice made with or_set_q.  Built with
 * -ffp-contract=off: no fused multiply-adds, so every product and sum is
 * rounded as written.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#define NVMAX 4         /* largest Q, nodes per axis */
#define NKMAX 16        /* largest Q*Q, populations */
#define NG 3            /* ghost layers: the WENO-5 stencil reaches 3 cells */

/* advection schemes (Sec. III.E) */
enum { OR_WENO5 = 0, OR_U1 = 1, OR_U2 = 2, OR_U3 = 3 };

int or_version(void) { return 2; }

/* The quadrature order Q of the model (3: D2Q9, 4: D2Q16). */
static int NV = 4, NK = 16;

/* ---------------------------------------------------------------------- */
/* Sec. III.A: probabilists' Hermite polynomials, eq. (hermite_polynomials)
 * in 1-D, by the three-term recurrence H_{n+1} = x H_n - n H_{n-1}.       */
double or_hermite(int n, double x)
{
    if (n < 0) return 0.0;
    double hm1 = 1.0, h = x;
    if (n == 0) return 1.0;
    for (int m = 1; m < n; ++m) {
        double hp1 = x * h - (double)m * hm1;
        hm1 = h;
        h = hp1;
    }
    return h;
}

static double factorial(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= (double)i;
    return r;
}

/* Nodes: roots of H_Q (Fig. stencils), ascending.  Q = 4: H_4(x) = x^4 -
 * 6x^2 + 3, x^2 = 3 -/+ sqrt(6) (App. A.2); Q = 3: H_3(x) = x^3 - 3x, x = 0,
 * +-sqrt(3) (App. A.1).  Weights eq. (GH_weights): w_k = Q! / H_{Q+1}(v_k)^2. */
void or_quadrature(double v[NVMAX], double w[NVMAX])
{
    if (NV == 4) {
        double a = sqrt(3.0 + sqrt(6.0));
        double b = sqrt(3.0 - sqrt(6.0));
        v[0] = -a; v[1] = -b; v[2] = b; v[3] = a;
    } else {
        v[0] = -sqrt(3.0); v[1] = 0.0; v[2] = sqrt(3.0);
    }
    for (int k = 0; k < NV; ++k) {
        double h = or_hermite(NV + 1, v[k]);
        w[k] = factorial(NV) / (h * h);
    }
}

/* Sec. III.C eq. (kernels):
 *   K_{k,k'}  = -w_k sum_{l=0}^{Q-1} H_{l+1}(v_k) H_l(v_k') / l!
 *   Kt_{k,k'} = -w_k sum_{l=0}^{Q-1} H_{l+1}(v_k) [H_{l+1}(v_k') + l H_{l-1}(v_k')] / l!
 * Row-major K[k*4 + k'].                                                  */
void or_kernels(double K[NKMAX], double Kt[NKMAX])
{
    double v[NVMAX], w[NVMAX];
    or_quadrature(v, w);
    for (int k = 0; k < NV; ++k)
        for (int kp = 0; kp < NV; ++kp) {
            double sk = 0.0, skt = 0.0;
            for (int l = 0; l < NV; ++l) {
                double a = or_hermite(l + 1, v[k]) / factorial(l);
                sk += a * or_hermite(l, v[kp]);
                skt += a * (or_hermite(l + 1, v[kp]) + (double)l * or_hermite(l - 1, v[kp]));
            }
            K[k * NV + kp] = -w[k] * sk;
            Kt[k * NV + kp] = -w[k] * skt;
        }
}

/* Process-wide constant tables, built from the definitions above for the
 * current Q. */
static double g_v[NVMAX], g_w1[NVMAX], g_K[NKMAX], g_Kt[NKMAX];
static int g_ready = 0;

static void tables(void)
{
    if (g_ready) return;
    or_quadrature(g_v, g_w1);
    or_kernels(g_K, g_Kt);
    g_ready = 1;
}

int or_set_q(int q)
{
    if (q != 3 && q != 4) return -1;
    NV = q;
    NK = q * q;
    g_ready = 0;
    tables();
    return 0;
}

int or_get_q(void) { return NV; }

/* ---------------------------------------------------------------------- */
/* Sec. III.B, eq. (feq_Q=4): isothermal equilibrium (T0 = 1)
 *   f^eq_k = n w_k [1 + v.u + ((v.u)^2 - u^2)/2 + v.u((v.u)^2 - 3u^2)/6]
 * and for Q = 3 eq. (feq_Q=3), the same without the cubic term.
 * With T != 1 the order-2 and order-3 Hermite coefficients gain the thermal
 * parts n(T-1)delta and n(T-1)(u delta)_sym, which add
 *   (T-1)(|v|^2 - 2)/2  and  v.u (T-1)(|v|^2 - 4)/2
 * inside the bracket (used for initial states only; Q = 3 keeps the first).  */
void or_feq_thermal(double n, double ut, double up, double T, double feq[NKMAX])
{
    tables();
    double u2 = ut * ut + up * up;
    double dT = T - 1.0;
    for (int kt = 0; kt < NV; ++kt)
        for (int kp = 0; kp < NV; ++kp) {
            double vt = g_v[kt], vp = g_v[kp];
            double vu = vt * ut + vp * up;
            double v2 = vt * vt + vp * vp;
            double br = 1.0 + vu + 0.5 * (vu * vu - u2 + dT * (v2 - 2.0));
            if (NV == 4) br += vu * (vu * vu - 3.0 * u2 + 3.0 * dT * (v2 - 4.0)) / 6.0;
            feq[kt * NV + kp] = n * g_w1[kt] * g_w1[kp] * br;
        }
}

/* Eq. (f_moments_sum): n = sum f, n u = sum f v. */
static void moments(const double f[NKMAX], double* n, double* ut, double* up)
{
    double s0 = 0.0, st = 0.0, sp = 0.0;
    for (int kt = 0; kt < NV; ++kt)
        for (int kp = 0; kp < NV; ++kp) {
            double x = f[kt * NV + kp];
            s0 += x;
            st += x * g_v[kt];
            sp += x * g_v[kp];
        }
    *n = s0;
    *ut = st / s0;
    *up = sp / s0;
}

/* BGK, Sec. III.B: C_k = -(f_k - f^eq_k)/tau, f^eq at the local n, u, T0 = 1. */
void or_collision(const double f[NKMAX], double tau, double C[NKMAX])
{
    tables();
    double n, ut, up, feq[NKMAX];
    moments(f, &n, &ut, &up);
    or_feq_thermal(n, ut, up, 1.0, feq);
    for (int k = 0; k < NK; ++k) C[k] = -(f[k] - feq[k]) / tau;
}

/* Inertial force, second term of eq. (Lf):
 *   G_k = -(cos th/(R sin th)) [ v_{kp}^2 (df/dv_th)_k - v_{kt} (d(f v_ph)/dv_ph)_k ]
 * with (df/dv_th)_{kt,kp} = sum_{b} K_{kt,b} f_{b,kp} and
 *      (d(f v_ph)/dv_ph)_{kt,kp} = sum_{b} Kt_{kp,b} f_{kt,b}   (eqs. (df)). */
void or_force(const double f[NKMAX], double theta, double R, double G[NKMAX])
{
    tables();
    double cotr = cos(theta) / (R * sin(theta));
    for (int kt = 0; kt < NV; ++kt)
        for (int kp = 0; kp < NV; ++kp) {
            double dfdvt = 0.0, dfvdvp = 0.0;
            for (int b = 0; b < NV; ++b) {
                dfdvt += g_K[kt * NV + b] * f[b * NV + kp];
                dfvdvp += g_Kt[kp * NV + b] * f[kt * NV + b];
            }
            double vt = g_v[kt], vp = g_v[kp];
            G[kt * NV + kp] = -cotr * (vp * vp * dfdvt - vt * dfvdvp);
        }
}

/* ---------------------------------------------------------------------- */
/* Sec. III.E: WENO-5 interface flux for a positive advection velocity.
 * Inputs are the five stencil points s-2 .. s+2 of the interface s+1/2:
 * h[] the flux function V f at each point, f[] the populations that enter
 * the smoothness indicators.                                              */
static double weno5_pos(const double h[5], const double f[5], double eps)
{
    /* eq. (fluxes_W5): candidate interpolants (V f already in h) */
    double F1 = h[0] / 3.0 - 7.0 * h[1] / 6.0 + 11.0 * h[2] / 6.0;
    double F2 = -h[1] / 6.0 + 5.0 * h[2] / 6.0 + h[3] / 3.0;
    double F3 = h[2] / 3.0 + 5.0 * h[3] / 6.0 - h[4] / 6.0;
    /* eq. (WENO5_sigma): smoothness functions of f */
    double a1 = f[0] - 2.0 * f[1] + f[2], b1 = f[0] - 4.0 * f[1] + 3.0 * f[2];
    double a2 = f[1] - 2.0 * f[2] + f[3], b2 = f[1] - f[3];
    double a3 = f[2] - 2.0 * f[3] + f[4], b3 = 3.0 * f[2] - 4.0 * f[3] + f[4];
    double s1 = 13.0 / 12.0 * a1 * a1 + 0.25 * b1 * b1;
    double s2 = 13.0 / 12.0 * a2 * a2 + 0.25 * b2 * b2;
    double s3 = 13.0 / 12.0 * a3 * a3 + 0.25 * b3 * b3;
    /* eq. (WENO5_delta) ideal weights; normalised nonlinear weights */
    double w1 = 0.1 / ((eps + s1) * (eps + s1));
    double w2 = 0.6 / ((eps + s2) * (eps + s2));
    double w3 = 0.3 / ((eps + s3) * (eps + s3));
    double ws = w1 + w2 + w3;
    return (w1 / ws) * F1 + (w2 / ws) * F2 + (w3 / ws) * F3;
}

/* Interface flux from the six points s-2 .. s+3 around s+1/2 (index 0 is
 * s-2).  dir > 0: upwind from the left (points s-2..s+2); dir < 0: the mirror
 * stencil (s+m -> s+1-m, i.e. points s+3, s+2, s+1, s, s-1).              */
double or_weno5(const double h6[6], const double f6[6], int dir, double eps)
{
    if (dir > 0) return weno5_pos(h6, f6, eps);
    double hm[5] = {h6[5], h6[4], h6[3], h6[2], h6[1]};
    double fm[5] = {f6[5], f6[4], f6[3], f6[2], f6[1]};
    return weno5_pos(hm, fm, eps);
}

/* Eq. (fluxes_U1-3) for a positive velocity from the points s-1, s, s+1 of
 * the interface s+1/2 (h already holds V f):
 *   U1: h_s;  U2: 3/2 h_s - 1/2 h_{s-1};  U3: 1/3 h_{s+1} + 5/6 h_s - 1/6 h_{s-1}. */
static double upwind_pos(int scheme, double hm1, double h0, double hp1)
{
    switch (scheme) {
    case OR_U1: return h0;
    case OR_U2: return 1.5 * h0 - 0.5 * hm1;
    default: return hp1 / 3.0 + 5.0 * h0 / 6.0 - hm1 / 6.0;
    }
}

/* Interface flux of any scheme from the six points s-2 .. s+3 (as or_weno5). */
double or_flux(int scheme, const double h6[6], const double f6[6], int dir, double eps)
{
    if (scheme == OR_WENO5) return or_weno5(h6, f6, dir, eps);
    if (dir > 0) return upwind_pos(scheme, h6[1], h6[2], h6[3]);
    return upwind_pos(scheme, h6[4], h6[3], h6[2]);   /* mirror: s+m -> s+1-m */
}

/* ---------------------------------------------------------------------- */
/* Ghost-extended copy of one population set, Sec. III.F.                   */
typedef struct {
    int nt, np, et, ep;   /* interior and extended sizes */
    double* g;            /* [16][nt+6][np+6] */
} ext_t;

static inline double* E(const ext_t* x, int k, int s, int q)
{
    return x->g + ((size_t)k * x->et + (size_t)(s + NG)) * x->ep + (size_t)(q + NG);
}

static void fill_ghosts(const double* f, ext_t* x)
{
    int nt = x->nt, np = x->np;
    /* interior */
    for (int k = 0; k < NK; ++k)
        for (int s = 0; s < nt; ++s)
            for (int q = 0; q < np; ++q)
                *E(x, k, s, q) = f[((size_t)k * nt + s) * np + q];
    /* eq. (bcs_theta): f(-dth, phi; v) = f(dth, phi + pi; -v), same at the
     * south pole.  Ghost row -m mirrors row m-1, ghost row nt-1+m mirrors row
     * nt-m, both at column q + np/2 and population 15-k (v -> -v).          */
    for (int k = 0; k < NK; ++k) {
        int kbar = NK - 1 - k;
        for (int m = 1; m <= NG; ++m)
            for (int q = 0; q < np; ++q) {
                int qp = (np == 1) ? q : (q + np / 2) % np;
                *E(x, k, -m, q) = f[((size_t)kbar * nt + (m - 1)) * np + qp];
                *E(x, k, nt - 1 + m, q) = f[((size_t)kbar * nt + (nt - m)) * np + qp];
            }
    }
    /* eq. (bcs_phi): periodic in phi, for every (also ghost) row */
    for (int k = 0; k < NK; ++k)
        for (int s = -NG; s < nt + NG; ++s)
            for (int m = 1; m <= NG; ++m) {
                *E(x, k, s, -m) = *E(x, k, s, ((np - m) % np + np) % np);
                *E(x, k, s, np - 1 + m) = *E(x, k, s, (m - 1) % np);
            }
}

/* ---------------------------------------------------------------------- */
/* Eq. (Lf) on the whole grid.
 *   L_k = -[ (F^th_{s+1/2} - F^th_{s-1/2})/dth + (F^ph_{q+1/2} - F^ph_{q-1/2})/dph ] / (R sin th_s)
 *         + G_k (inertial force) + C_k (BGK)
 * with the theta flux function V f = v sin(theta_j) f_j.  With komissarov != 0
 * the theta part is eq. (Komissarov_scheme) instead:
 *   [F^th_{s+1/2} sin th_{s+1/2} - F^th_{s-1/2} sin th_{s-1/2}] / (R (cos th_{s-1/2} - cos th_{s+1/2}))
 * with V f = v f_j and the interface angles of eq. (Komissarov_sin_cos)
 * (0-based: th_{s+1/2} = (s+1) dth).
 * fn / fs (optional, [16][np]) receive the theta fluxes through the first
 * (north, s = -1/2) and last (south, s = nt-1/2) interfaces, as they enter the
 * theta difference (times sin th_{-1/2} = 0 and sin th_{nt-1/2} = 0 for the
 * Komissarov form).                                                        */
static int rhs_ext(int nt, int np, double R, double tau, double eps, int scheme, int komissarov,
                   const double* f, double* L, double* fn, double* fs, int nthreads)
{
    tables();
    ext_t x;
    x.nt = nt; x.np = np; x.et = nt + 2 * NG; x.ep = np + 2 * NG;
    x.g = (double*)malloc(sizeof(double) * NK * (size_t)x.et * x.ep);
    /* interface fluxes: theta [16][nt+1][np], phi [16][nt][np+1] */
    double* Ft = (double*)malloc(sizeof(double) * NK * (size_t)(nt + 1) * np);
    double* Fp = (double*)malloc(sizeof(double) * NK * (size_t)nt * (np + 1));
    if (!x.g || !Ft || !Fp) { free(x.g); free(Ft); free(Fp); return -1; }
    fill_ghosts(f, &x);

    const double pi = acos(-1.0);
    const double dth = pi / nt, dph = 2.0 * pi / np;
    (void)nthreads;

    /* theta fluxes at s+1/2, s = -1 .. nt-1 */
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int s = -1; s < nt; ++s) {
        double h6[6], f6[6];
        for (int k = 0; k < NK; ++k) {
            double vk = g_v[k / NV];
            int dir = vk > 0.0 ? 1 : -1;
            for (int q = 0; q < np; ++q) {
                for (int m = 0; m < 6; ++m) {
                    int j = s - 2 + m;
                    double sj = komissarov ? 1.0 : sin((j + 0.5) * dth);   /* signed in ghost rows */
                    f6[m] = *E(&x, k, j, q);
                    h6[m] = vk * sj * f6[m];
                }
                double F = or_flux(scheme, h6, f6, dir, eps);
                /* sin th_{s+1/2} = sin((s+1) dth), written as the sine of the
                 * angle to the nearer pole so that both pole values are 0 */
                if (komissarov) F *= sin((s + 1 < nt - (s + 1) ? s + 1 : nt - (s + 1)) * dth);
                Ft[((size_t)k * (nt + 1) + (s + 1)) * np + q] = F;
            }
        }
    }
    /* phi fluxes at q+1/2, q = -1 .. np-1 */
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int s = 0; s < nt; ++s) {
        double h6[6], f6[6];
        for (int k = 0; k < NK; ++k) {
            double vk = g_v[k % NV];
            int dir = vk > 0.0 ? 1 : -1;
            for (int q = -1; q < np; ++q) {
                for (int m = 0; m < 6; ++m) {
                    f6[m] = *E(&x, k, s, q - 2 + m);
                    h6[m] = vk * f6[m];
                }
                Fp[((size_t)k * nt + s) * (np + 1) + (q + 1)] = or_flux(scheme, h6, f6, dir, eps);
            }
        }
    }
    /* assemble L */
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int s = 0; s < nt; ++s) {
        double th = (s + 0.5) * dth;
        double rs = R * sin(th);
        double rk = R * (cos(s * dth) - cos((s + 1) * dth));   /* Komissarov band */
        double fc[NKMAX], C[NKMAX], G[NKMAX];
        for (int q = 0; q < np; ++q) {
            for (int k = 0; k < NK; ++k) fc[k] = *E(&x, k, s, q);
            or_collision(fc, tau, C);
            or_force(fc, th, R, G);
            for (int k = 0; k < NK; ++k) {
                double ftp = Ft[((size_t)k * (nt + 1) + (s + 1)) * np + q];
                double ftm = Ft[((size_t)k * (nt + 1) + s) * np + q];
                double fpp = Fp[((size_t)k * nt + s) * (np + 1) + (q + 1)];
                double fpm = Fp[((size_t)k * nt + s) * (np + 1) + q];
                double adv = komissarov ? (ftp - ftm) / rk + (fpp - fpm) / (dph * rs)
                                        : ((ftp - ftm) / dth + (fpp - fpm) / dph) / rs;
                L[((size_t)k * nt + s) * np + q] = -adv + G[k] + C[k];
            }
        }
    }
    if (fn && fs)
        for (int k = 0; k < NK; ++k)
            for (int q = 0; q < np; ++q) {
                fn[(size_t)k * np + q] = Ft[((size_t)k * (nt + 1) + 0) * np + q];
                fs[(size_t)k * np + q] = Ft[((size_t)k * (nt + 1) + nt) * np + q];
            }
    free(x.g); free(Ft); free(Fp);
    return 0;
}

static int check_grid(int nt, int np)
{
    if (nt < NG || np < 1) return -1;
    if (np > 1 && (np % 2) != 0) return -1;  /* phi + pi must be a grid column */
    return 0;
}

int or_rhs_s(int nt, int np, double R, double tau, double eps, int scheme, int komissarov,
             const double* f, double* L, double* flux_north, double* flux_south, int nthreads)
{
    if (check_grid(nt, np) || scheme < OR_WENO5 || scheme > OR_U3) return -1;
    return rhs_ext(nt, np, R, tau, eps, scheme, komissarov, f, L, flux_north, flux_south, nthreads);
}

int or_rhs(int nt, int np, double R, double tau, double eps, const double* f,
           double* L, double* flux_north, double* flux_south, int nthreads)
{
    return or_rhs_s(nt, np, R, tau, eps, OR_WENO5, 0, f, L, flux_north, flux_south, nthreads);
}

/* Sec. III.G: one SSP-RK3 step per iteration,
 *   f1 = f + dt L[f]
 *   f2 = 3/4 f + 1/4 f1 + 1/4 dt L[f1]
 *   f' = 1/3 f + 2/3 f2 + 2/3 dt L[f2]
 * budget (optional) accumulates, over the steps, the mass change that the
 * pole fluxes imply: dt * sum over stages with weights (1/6, 1/6, 2/3) of
 *   -R dph sum_{k,q} (F^th_{nt-1/2} - F^th_{-1/2}).                        */
int or_step_s(int nt, int np, double R, double tau, double dt, double eps, int scheme,
              int komissarov, double* f, int64_t nsteps, int nthreads, double* budget)
{
    if (check_grid(nt, np) || scheme < OR_WENO5 || scheme > OR_U3) return -1;
    size_t n = (size_t)NK * nt * np;
    double* L = (double*)malloc(sizeof(double) * n);
    double* f1 = (double*)malloc(sizeof(double) * n);
    double* f2 = (double*)malloc(sizeof(double) * n);
    double* fn = (double*)malloc(sizeof(double) * NK * (size_t)np);
    double* fs = (double*)malloc(sizeof(double) * NK * (size_t)np);
    if (!L || !f1 || !f2 || !fn || !fs) {
        free(L); free(f1); free(f2); free(fn); free(fs);
        return -1;
    }
    const double dph = 2.0 * acos(-1.0) / np;
    const double stage_w[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
    int rc = 0;
    for (int64_t it = 0; it < nsteps && rc == 0; ++it) {
        double b[3] = {0.0, 0.0, 0.0};
        const double* in[3] = {f, f1, f2};
        for (int st = 0; st < 3 && rc == 0; ++st) {
            rc = rhs_ext(nt, np, R, tau, eps, scheme, komissarov, in[st], L, fn, fs, nthreads);
            if (rc) break;
            if (budget) {
                double acc = 0.0;
                for (size_t i = 0; i < (size_t)NK * np; ++i) acc += fs[i] - fn[i];
                b[st] = -R * dph * acc;
            }
            if (st == 0) {
                for (size_t i = 0; i < n; ++i) f1[i] = f[i] + dt * L[i];
            } else if (st == 1) {
                for (size_t i = 0; i < n; ++i)
                    f2[i] = 0.75 * f[i] + 0.25 * f1[i] + 0.25 * dt * L[i];
            } else {
                for (size_t i = 0; i < n; ++i)
                    f[i] = f[i] / 3.0 + 2.0 * f2[i] / 3.0 + 2.0 * dt * L[i] / 3.0;
            }
        }
        if (budget && rc == 0)
            *budget += dt * (stage_w[0] * b[0] + stage_w[1] * b[1] + stage_w[2] * b[2]);
    }
    free(L); free(f1); free(f2); free(fn); free(fs);
    return rc;
}

int or_step(int nt, int np, double R, double tau, double dt, double eps,
            double* f, int64_t nsteps, int nthreads, double* budget)
{
    return or_step_s(nt, np, R, tau, dt, eps, OR_WENO5, 0, f, nsteps, nthreads, budget);
}

/* ---------------------------------------------------------------------- */
/* Initial populations: f_k = f^eq_k(rho, u, T) per cell (T NULL: T = 1).  */
int or_init(int nt, int np, const double* rho, const double* ut, const double* up,
            const double* T, double* f)
{
    if (check_grid(nt, np)) return -1;
    double feq[NKMAX];
    for (int s = 0; s < nt; ++s)
        for (int q = 0; q < np; ++q) {
            size_t c = (size_t)s * np + q;
            or_feq_thermal(rho[c], ut[c], up[c], T ? T[c] : 1.0, feq);
            for (int k = 0; k < NK; ++k) f[((size_t)k * nt + s) * np + q] = feq[k];
        }
    return 0;
}

/* Macroscopic fields, eq. (f_moments_sum); T = sum f |v-u|^2 / (2 n). */
int or_moments(int nt, int np, const double* f, double* rho, double* ut,
               double* up, double* T)
{
    if (check_grid(nt, np)) return -1;
    tables();
    double fc[NKMAX];
    for (int s = 0; s < nt; ++s)
        for (int q = 0; q < np; ++q) {
            size_t c = (size_t)s * np + q;
            for (int k = 0; k < NK; ++k) fc[k] = f[((size_t)k * nt + s) * np + q];
            double n, a, b;
            moments(fc, &n, &a, &b);
            rho[c] = n; ut[c] = a; up[c] = b;
            if (T) {
                double e = 0.0;
                for (int kt = 0; kt < NV; ++kt)
                    for (int kp = 0; kp < NV; ++kp) {
                        double dt_ = g_v[kt] - a, dp_ = g_v[kp] - b;
                        e += fc[kt * NV + kp] * (dt_ * dt_ + dp_ * dp_);
                    }
                T[c] = e / (2.0 * n);
            }
        }
    return 0;
}

/* Vorticity omega = [d_th(u_ph sin th) - d_ph u_th] / (R sin th) (Sec. IV.D),
 * fourth-order central differences.  Across a pole the velocity changes sign
 * (v -> -v at phi + pi) while sin th changes sign too, so u_ph sin th
 * continues evenly to column q + np/2.                                     */
int or_vorticity(int nt, int np, double R, const double* ut, const double* up,
                 double* om)
{
    if (check_grid(nt, np)) return -1;
    const double pi = acos(-1.0);
    const double dth = pi / nt, dph = 2.0 * pi / np;
    for (int s = 0; s < nt; ++s)
        for (int q = 0; q < np; ++q) {
            double g[5];
            for (int m = -2; m <= 2; ++m) {
                int j = s + m, qq = q;
                if (j < 0 || j >= nt) {
                    qq = (np == 1) ? q : (q + np / 2) % np;
                    j = (j < 0) ? (-1 - j) : (2 * nt - 1 - j);
                }
                g[m + 2] = up[(size_t)j * np + qq] * sin((j + 0.5) * dth);
            }
            double dg = (g[0] - 8.0 * g[1] + 8.0 * g[3] - g[4]) / (12.0 * dth);
            double du = 0.0;
            if (np > 1) {
                double u[5];
                for (int m = -2; m <= 2; ++m)
                    u[m + 2] = ut[(size_t)s * np + (size_t)(((q + m) % np + np) % np)];
                du = (u[0] - 8.0 * u[1] + 8.0 * u[3] - u[4]) / (12.0 * dph);
            }
            om[(size_t)s * np + q] = (dg - du) / (R * sin((s + 0.5) * dth));
        }
    return 0;
}

/* Global FP64 diagnostics (area element R^2 sin th dth dph):
 *   out[0] mass, out[1] kinetic-theory energy sum f|v|^2/2, out[2] kinetic
 *   energy rho|u|^2/2, out[3] angular momentum rho u_ph R sin th,
 *   out[4] number of non-finite populations, out[5] max |u|,
 *   out[6] min rho, out[7] max rho.                                         */
int or_diagnostics(int nt, int np, double R, const double* f, double out[8])
{
    if (check_grid(nt, np)) return -1;
    tables();
    const double pi = acos(-1.0);
    const double dth = pi / nt, dph = 2.0 * pi / np;
    double M = 0.0, Et = 0.0, Ek = 0.0, Lz = 0.0, nbad = 0.0, umax = 0.0;
    double rmin = INFINITY, rmax = -INFINITY;
    for (int s = 0; s < nt; ++s) {
        double st = sin((s + 0.5) * dth);
        double dA = R * R * st * dth * dph;
        for (int q = 0; q < np; ++q) {
            double fc[NKMAX], e = 0.0;
            for (int k = 0; k < NK; ++k) {
                fc[k] = f[((size_t)k * nt + s) * np + q];
                if (!isfinite(fc[k])) nbad += 1.0;
                e += 0.5 * fc[k] * (g_v[k / NV] * g_v[k / NV] + g_v[k % NV] * g_v[k % NV]);
            }
            double n, a, b;
            moments(fc, &n, &a, &b);
            double u = sqrt(a * a + b * b);
            M += dA * n;
            Et += dA * e;
            Ek += dA * 0.5 * n * (a * a + b * b);
            Lz += dA * n * b * R * st;
            if (u > umax) umax = u;
            if (n < rmin) rmin = n;
            if (n > rmax) rmax = n;
        }
    }
    out[0] = M; out[1] = Et; out[2] = Ek; out[3] = Lz;
    out[4] = nbad; out[5] = umax; out[6] = rmin; out[7] = rmax;
    return 0;
}

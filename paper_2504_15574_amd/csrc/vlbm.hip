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

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/vlbm.h"

namespace {

constexpr int NQMAX = 4;    // nodes per axis (Q = 3: D2Q9, Q = 4: D2Q16)
constexpr int NKMAX = 16;   // populations Q * Q
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
// (arrays packed with the stride Q of the model: k = Q kt + kp)
struct Consts {
    int q;                    // quadrature order Q (3 or 4)
    double v[NQMAX];          // ascending Gauss-Hermite nodes (roots of H_Q)
    double wk[NKMAX];         // product weights w_k
    double K[NKMAX];          // K^H,  row k, column k'
    double Kt[NKMAX];         // K~^H
    double scale[NKMAX];      // FP16 storage scale 2^e_k (1 for the other formats)
    double iscale[NKMAX];     // 1 / scale
};

// per-row tables in the workspace (FP64)
struct Rows {
    const double* sinv;      // [nt + 6]: sin((j + 1/2) dth), j = -3 .. nt+2 (signed)
    const double* inv_sdth;  // [nt]: 1 / (R sin th_s dth)
    const double* inv_sdph;  // [nt]: 1 / (R sin th_s dph)
    const double* cot;       // [nt]: cos th_s / (R sin th_s)
    const double* rest;      // [16][nt]: dt * L of the rest state w_k rho0 at central-candidate weights
    const double* dC;        // [2][nt + 1][2]: rho0 (C1 - C2), rho0 (C3 - C2) of sin th per interface
    const double* sI;        // [nt + 1]: factor of the theta flux at interface i (Komissarov: sin th_{i-1/2})
};

// the constants the stage kernel uses, in its arithmetic type
template <class T>
struct ConstsT {
    T v[NQMAX], wk[NKMAX], scale[NKMAX], iscale[NKMAX];
    // weight of the rest state's theta flux per unit node speed: w_k in FP64; in
    // FP32 v_k w_k (FP64 node and weight) over the FP32 node, so that the speed
    // factor times it reproduces the FP64 product the rest-state tables use
    T wr[NKMAX];
    T K[NKMAX], Kt[NKMAX];   // the force kernels K^H, K~^H (row-major, stride Q)
    T nv2[NQMAX];            // -v^2 per node
    // equilibrium coefficients that make its mass and momentum exact on the
    // rule's own moments S2 = sum w v^2, S4 = sum w v^4, S22 = sum w vt^2 vp^2
    T eq_e1;    // 1/S2 - 1 (extra weight of the linear term)
    T eq_hb;    // -S2/2 (u^2 coefficient of the quadratic term)
    T eq_g6;    // (S4 + 3 S22)/(12 S2) (u^2 coefficient of the cubic term)
};

// Per-row constants of the stage kernel in its arithmetic type, computed on the
// host from the run's dt and velocity nodes (v_o, v_i: the outer and inner
// node magnitudes; the inner node is 0 for Q = 3).  The WENO-5 variants divide
// the theta and phi factors by 6 (their fluxes arrive scaled by 6).
template <class T>
struct CellRowK {       // cell row s
    T th_o, th_i;       // v_o, v_i times dt / (R sin th_s dth) (Komissarov: dt / (R (cos - cos)))
    T ph_o, ph_i;       // v_o, v_i times dt / (R sin th_s dph)
    T dtcot;            // dt cot(th_s) / R
    T pad[3];
};
template <class T>
struct FaceRowK {       // theta interface i (between rows i-1 and i)
    T cp1, cp3;         // 3 and 6 times the rest state's C1 - C2, C3 - C2 (v > 0)
    T cm1, cm3;         // the same on the mirrored stencil (v < 0)
    T sI;               // factor of the theta flux (Komissarov: sin th at the interface, else 1)
    T pad[3];
};
// SSP-RK3 (Sec. III.G): stage i writes a_i g_n + b_i (g_in + dt L(g_in))
constexpr double RK_A[3] = {0.0, 0.75, 1.0 / 3.0}, RK_B[3] = {1.0, 0.25, 2.0 / 3.0};
// (per-stage launches compile stage 1 without g_n and stages 2, 3 with it)
static_assert(RK_A[0] == 0.0 && RK_A[1] != 0.0 && RK_A[2] != 0.0, "only stage 1 skips g_n");
// run constants in both arithmetic types (uniform per workgroup: scalar loads)
enum { U_DTI, U_EPSK, U_OMDTI, U_RHO0, U_A, U_B, U_N };

// One run (context) at one RK stage, in device memory inside the context's
// workspace; written once at creation.
struct RunDesc {
    const void* gin;      // stage input (halo reads)
    const void* gn;       // f_n deviations (point reads), may alias out
    void* out;            // stage output
    Rows rows;
    const float* rest_f;  // rest[] times this stage's b, in FP32, for the float kernels
    const float* sinv_f;  // Rows::sinv rounded to FP32, for the float kernels
    int nt, np;
    double dt, inv_tau, rho0, eps;
    double a, b;          // out = a g_n + b (g_in + dt L)
    const uint32_t* ctr;  // completed steps (reduced-precision storage: dither phase)
    uint32_t seq;         // 16 * (stage - 1)
    int scheme;           // VLBM_ADV_WENO5 / U1 / U2 / U3
    const void* rowk;     // CellRowK<T>[nt] of the storage's arithmetic type (float: times b)
    const void* facek;    // FaceRowK<T>[nt + 1]
    // dt/tau, 12/13 eps (the scaled WENO epsilon), 1 - dt/tau, rho0, a, b;
    // uf[U_DTI] is b dt/tau (the float kernels fold b into the increment)
    double ud[U_N];
    float uf[U_N];
};
template <class T> __device__ __forceinline__ T uni(const RunDesc& D, int i);
template <> __device__ __forceinline__ double uni<double>(const RunDesc& D, int i) { return D.ud[i]; }
template <> __device__ __forceinline__ float uni<float>(const RunDesc& D, int i) { return D.uf[i]; }

// Kernel arguments of a stage launch over the tiles of up to MAXRUNS runs
// sharing one storage format (one run for vlbm_step).
constexpr int MAXRUNS = 64;
struct StageArgs {
    ConstsT<double> cd;
    ConstsT<float> cf;
    RunDesc run0;                  // the run of a single-run launch, by value
    int nruns;
    int tile_start[MAXRUNS + 1];   // prefix sums of the runs' tile counts
    const RunDesc* desc[MAXRUNS];
};

// ---------------------------------------------------------------------------
// storage formats.  ld/st address flat memory; bld/bst go through a buffer
// resource (one 32-bit per-lane byte offset plus a wave-uniform scalar byte
// offset), which keeps 64-bit address arithmetic out of the stage kernel.
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    // word 3 = 0x00020000: raw (untyped) 32-bit buffer access on gfx9-family parts
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

struct StF64 {
    using S = double;
    using T = double;
    static constexpr int B = 8;
    __device__ static T rload(rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    __device__ static T ld(const S* p, size_t i, double) { return p[i]; }
    __device__ static void st(S* p, size_t i, T v, double) { p[i] = v; }
    __device__ static T bld(rsrc_t r, uint32_t vo, uint32_t so, float) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    __device__ static void bst(rsrc_t r, uint32_t vo, uint32_t so, T v, float) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, vo, so, 0);
    }
};
struct StF32 {
    using S = float;
    using T = float;
    static constexpr int B = 4;
    __device__ static T rload(rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    __device__ static T ld(const S* p, size_t i, double) { return p[i]; }
    __device__ static void st(S* p, size_t i, T v, double) { p[i] = v; }
    __device__ static T bld(rsrc_t r, uint32_t vo, uint32_t so, float) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    __device__ static void bst(rsrc_t r, uint32_t vo, uint32_t so, T v, float) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
    }
    // store g + d rounded with a dither x * 2^-32 ulp(g), x in [-2^31, 2^31):
    // ulp(g) = 2^(E - 150) for the biased exponent E of g, so the dither is x
    // times 2^(E - 182), the float whose exponent field is E - 55 (a saturating
    // subtraction: |g| < 2^-72 gets no dither)
    __device__ static void bst_dither(rsrc_t r, uint32_t vo, uint32_t so, T g, T d, float x, float) {
        const uint32_t eb = __builtin_bit_cast(uint32_t, g) & 0x7f800000u;
        const float s = __builtin_bit_cast(float, __builtin_elementwise_sub_sat(eb, 55u << 23));
        const T v = g + fma(x, s, d);
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
    }
};
struct StF16 {
    using S = _Float16;
    using T = float;
    static constexpr int B = 2;
    __device__ static T rload(rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    __device__ static T ld(const S* p, size_t i, double isc) { return (float)p[i] * (float)isc; }
    __device__ static void st(S* p, size_t i, T v, double sc) { p[i] = (_Float16)(v * (float)sc); }
    __device__ static T bld(rsrc_t r, uint32_t vo, uint32_t so, float isc) {
        return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0)) * isc;
    }
    __device__ static void bst(rsrc_t r, uint32_t vo, uint32_t so, T v, float sc) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)(v * sc)), r, vo, so, 0);
    }
    // the FP16 ulp of the scaled value y is 2^(E - 137) for biased FP32 exponent
    // E >= 113 and 2^-24 below (FP16 subnormals); the dither is x * 2^-32 of it
    __device__ static void bst_dither(rsrc_t r, uint32_t vo, uint32_t so, T g, T d, float x, float sc) {
        const T y = (g + d) * sc;
        int E = (int)((__builtin_bit_cast(uint32_t, y) >> 23) & 0xffu);
        E = E < 113 ? 113 : E;
        const T v = y + __builtin_ldexpf(x, E - 169);
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r, vo, so, 0);
    }
};

// ---------------------------------------------------------------------------
// WENO-5 interface flux for an upwind direction, eqs. (fluxes_W5), (WENO5_delta),
// (WENO5_sigma), from the five stencil points in upwind order (s-2 .. s+2 for a
// positive velocity, the mirror s+3 .. s-1 for a negative one).  h: flux
// function at the points; g: the values of the smoothness indicators (a
// deviation from a uniform state gives the same indicators).
//   F = F2 + w1 (F1 - F2) + w3 (F3 - F2),  w_i = (d_i / q_i) / sum_j (d_j / q_j),
//   q_i = (eps + sigma_i)^2,  d = (1, 6, 3) / 10.
// Returned scaled by 6 (the caller folds 1/6 into its flux-difference factor):
//   6F = G2 + q2 (q3 A + 1.5 q1 B) / [q2 (q3 / 2 + 1.5 q1) + 3 q1 q3]
// with G2 = 6 F2, A = 3 (F1 - F2), B = 6 (F3 - F2); multiplying numerator and
// denominator of the weights by q1 q2 q3 needs a single reciprocal.  The
// indicators are carried as a^2 + (3/13) b^2 (12/13 of sigma, with eps scaled
// to match), which leaves the normalised weights unchanged.  REST: wr c1 and
// wr c3 add the rest state's candidate differences, which share the weights
// (theta direction; c1, c3 arrive scaled by 3 and 6; wr is the rest weight per
// unit speed, since the caller multiplies the flux difference by the speed).
template <class T> __device__ __forceinline__ T rcp_(T x);
template <> __device__ __forceinline__ float rcp_<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp_<double>(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);      // one Newton step on the hardware estimate
    return fma(r, e, r);
}
// 1/x with one Newton step in either type: the hardware FP32 estimate alone is
// not correctly rounded, and a bias in 1/rho is a bias in u (a small force)
template <class T> __device__ __forceinline__ T rcp_nr(T x) {
    const T r = rcp_(x);
    return fma(r, fma(-x, r, T(1)), r);
}

// REST also marks the theta flux (h = sin th g); without it h is g itself
// (phi), and the candidate differences come from the indicators' second
// differences: 3 (h2 - h1) + (h0 - h3) = a1 - a2, 3 (h3 - h2) + (h1 - h4) =
// a2 - a3, 5 h2 + 2 h3 - h1 = 6 h2 + 2 D2 + D1 (one instruction fewer each for
// A and B).
template <class T, bool REST>
__device__ __forceinline__ T weno5x6(T h0, T h1, T h2, T h3, T h4, T g0, T g1, T g2, T g3, T g4,
                                     T epsk, T wr, T c1, T c3) {
    constexpr bool DIRECT = REST;
    T G2, A, B;
    if constexpr (DIRECT) {
        G2 = fma(T(5), h2, fma(T(2), h3, -h1));                 // 6 F2
        A = fma(T(3), h2 - h1, h0 - h3);                        // 3 (F1 - F2)
        B = fma(T(3), h3 - h2, h1 - h4);                        // 6 (F3 - F2)
        if constexpr (REST) {
            A = fma(wr, c1, A);
            B = fma(wr, c3, B);
        }
    }
    const T D0 = g1 - g0, D1 = g2 - g1, D2 = g3 - g2, D3 = g4 - g3;
    const T a1 = D1 - D0, a2 = D2 - D1, a3 = D3 - D2;
    if constexpr (!DIRECT) {
        G2 = fma(T(6), g2, fma(T(2), D2, D1));
        A = a1 - a2;
        B = a2 - a3;
    }
    const T b1 = fma(T(2), D1, a1), b2 = D1 + D2, b3 = fma(T(-2), D2, a3);
    const T e1 = fma(a1, a1, fma(T(3.0 / 13.0) * b1, b1, epsk));
    const T e2 = fma(a2, a2, fma(T(3.0 / 13.0) * b2, b2, epsk));
    const T e3 = fma(a3, a3, fma(T(3.0 / 13.0) * b3, b3, epsk));
    const T q1 = e1 * e1, q2 = e2 * e2, q3 = e3 * e3;
    const T u = T(1.5) * q1;
    const T den = fma(q2, fma(T(0.5), q3, u), (u + u) * q3);
    const T num = q2 * fma(u, B, q3 * A);
    return fma(num, rcp_(den), G2);
}

// Upwind fluxes U1, U2, U3 of eq. (fluxes_U1-3) from the stencil points in
// upwind order (a = s-1, b = s, c = s+1 for a positive velocity; the mirror
// s+2, s+1, s for a negative one).
// (written with explicit fma, so that every kernel rounds them the same way)
template <class T>
__device__ __forceinline__ T upwind(int scheme, T a, T b, T c) {
    if (scheme == VLBM_ADV_U1) return b;
    if (scheme == VLBM_ADV_U2) return fma(T(1.5), b, T(-0.5) * a);
    return fma(T(1.0 / 3.0), c, fma(T(5.0 / 6.0), b, T(-1.0 / 6.0) * a));
}

template <class T> __device__ __forceinline__ const ConstsT<T>& consts_of(const StageArgs& A);
template <> __device__ __forceinline__ const ConstsT<double>& consts_of<double>(const StageArgs& A) { return A.cd; }
template <> __device__ __forceinline__ const ConstsT<float>& consts_of<float>(const StageArgs& A) { return A.cf; }

__device__ __forceinline__ int wrap(int q, int np) {
    int r = q % np;
    return r < 0 ? r + np : r;
}
// the same for q in [-np, 2 np)
__device__ __forceinline__ int wrap1(int q, int np) {
    return q < 0 ? q + np : (q >= np ? q - np : q);
}

// ---------------------------------------------------------------------------
// Fused RK stage.
//
// Tile: 15 theta rows x 16 phi columns per 256-thread workgroup.  With this
// shape the 16 x 16 theta interfaces and the 15 x 17 phi interfaces of a tile
// are one WENO evaluation per thread each, so every interface flux is computed
// exactly once and exchanged through LDS.  Populations are processed one at a
// time; each population's tile with its 3-cell cross-shaped halo (pole rows
// gathered from column q + np/2 and population 15 - k, phi periodic) sits in a
// triple-buffered LDS slot, so the global loads of the next populations
// overlap the fluxes of population k and one barrier per population suffices.
// The 240
// cell threads accumulate dt*L for all 16 populations in registers, starting
// from the rest-state table: advection and the rank-1 updates of the inertial
// force (FP64 also -g/tau); the equilibrium is added at the end from the
// moments (FP64: running sums; float: sums of the 16 inputs kept in registers).
// Two tile shapes fit this thread mapping ((TS + 1) TQ theta interfaces = 256
// threads, at most two cross-shaped loads per thread): 15 x 16 (the default,
// least halo per cell) and 7 x 32 (fewer rows, for grids whose row count 15
// divides badly).  Neither changes any cell's arithmetic.
constexpr int NTHR = 256;
// D2Q16 populations (k = 4 k_theta + k_phi over ascending nodes) in rounds of
// four that share the signs of both speed components: v_theta < 0 for
// k_theta = 0, 1 and > 0 for 2, 3, likewise v_phi with k_phi.
constexpr int ROUND_ORDER[16] = {0, 1, 4, 5, 2, 3, 6, 7, 8, 9, 12, 13, 10, 11, 14, 15};
template <int TS_, int TQ_>
struct TileShape {
    static constexpr int TS = TS_, TQ = TQ_;
    static constexpr int LR = TS + 2 * NGH, LC = TQ + 2 * NGH, LT = LR * LC;
    static constexpr int NLOAD = LR * TQ + TS * 2 * NGH;       // cross-shaped values
    static constexpr int NFT = (TS + 1) * TQ;                  // theta interfaces
    static constexpr int NFP = TS * (TQ + 1);                  // phi interfaces
    static_assert(NFT == NTHR && NFP <= NTHR && NLOAD <= 2 * NTHR && TS * TQ <= NTHR, "tile shape");
};
// LDS placement of one tile slot, element (row r, column c) of the LR x LC
// cross-shaped tile.  A wave of the 15 x 16 tile reads four consecutive rows of
// 16 elements at once (lanes 16i..16i+15 take row r0 + i).  Row-major with pitch
// 22, rows r and r+1 share LDS banks for 4-byte values; so 4-byte slots keep the
// even rows in one block and the odd rows in another, each with pitch 32, the odd
// block starting 16 elements off modulo 32: the four rows then fill disjoint
// banks (32 or 64 banks of 4 bytes).  8-byte values (16 lanes per LDS cycle) and
// the 7 x 32 tile (32 lanes per row) keep the row-major layout.
template <class Tl, int BYTES>
struct SlotLayout {
    static constexpr bool SPLIT = BYTES == 4 && Tl::TQ == 16;
    static constexpr int OB = SPLIT ? ((Tl::LR + 1) / 2) * 32 + 16 : Tl::LC;   // row 1
    static constexpr int RS2 = SPLIT ? 32 : 2 * Tl::LC;                         // row r -> r + 2
    // last even row's end: the gap up to OB takes the unused load slots
    static constexpr int EVEN_END = ((Tl::LR - 1) >> 1) * 32 + Tl::LC;
    static_assert(!SPLIT || EVEN_END < OB, "slot layout");
    // elements per slot (past the last odd row) and where unused load slots write
    static constexpr int SIZE = SPLIT ? OB + ((Tl::LR - 2) >> 1) * 32 + Tl::LC : Tl::LT + (BYTES == 8 ? 1 : 8);
    static constexpr int DUMMY = SPLIT ? EVEN_END : Tl::LT;
    __device__ static int at(int r, int c) { return (r & 1) * OB + (r >> 1) * RS2 + c; }
};
using Tile15x16 = TileShape<15, 16>;
using Tile7x32 = TileShape<7, 32>;
constexpr int TILE_ROWS[2] = {15, 7}, TILE_COLS[2] = {16, 32};

__host__ __device__ inline int n_tiles(int nt, int np, int shape) {
    const int ts = shape ? 7 : 15, tq = shape ? 32 : 16;
    return ((nt + ts - 1) / ts) * ((np + tq - 1) / tq);
}

// VAR: 0 the WENO-5 standard form (the default; fewest registers), 1 WENO-5
// with the interface factor of the Komissarov form (or 1), 2 the upwind
// fluxes U1/U2/U3 (order read per run) with the interface factor.  A launch
// covers runs of one variant.
enum { VAR_WENO = 0, VAR_WENO_GEN = 1, VAR_UPWIND = 2 };
// Minimum waves per SIMD the register allocation must allow: 7 for the float
// kernels (at most 72 VGPRs; the general WENO-5 variant keeps two values in
// scratch across the population loop and still gains 3.7 % over 6 waves),
// 5 for FP64 (at most 96 VGPRs: its row factors in LDS, its populations
// loaded straight into LDS with nothing in flight in registers, 24 KB of LDS
// per workgroup).  Six FP64 waves fit (80 VGPRs) with barriers that wait for
// all direct loads, but the longer load overlap at five is faster.
template <class T, int VAR>
constexpr int stage_min_waves() { return sizeof(T) == 8 ? 5 : 7; }
// The float formats of D2Q16 with the WENO-5 standard form or an upwind
// scheme (either theta form) on 15 x 16 tiles run stage_tile_rounds (same
// bits as stage_tile).  FP64 stays on stage_tile:
// the rounds kernel needs 128 VGPRs there (four waves per SIMD, with spills;
// three waves without) and ran 25 % (8 %) slower than stage_tile at five.
template <class T, class Tl, int VAR, int NQ>
constexpr bool uses_rounds() {
    return sizeof(T) != 8 && Tl::TS == 15 && (VAR == VAR_WENO || VAR == VAR_UPWIND) && NQ == 4;
}
// minimum waves per SIMD of a stage launch (the rounds kernel: seven with
// direct-to-LDS loads, which hold nothing in registers, at most 72 VGPRs and
// 23 KB of LDS per workgroup; six, at most 80 VGPRs, when loading through
// registers: seven would spill)
template <class St, class Tl, int VAR, int NQ, bool LDSDMA>
constexpr int launch_min_waves() {
    return uses_rounds<typename St::T, Tl, VAR, NQ>() ? (LDSDMA ? 7 : 6) : stage_min_waves<typename St::T, VAR>();
}
// The end of a stage for one cell: BGK's equilibrium part from the cell's
// moments, the SSP-RK3 combination and the store in the storage format.  acc
// holds g + dt L without the equilibrium (FP64) or dt L without it (float
// formats, which keep the cell's stage input in gk); FP64 brings the moments
// of its running sums (drho, jt, jp), the float formats form them from gk.
// Stages 2 and 3 combine with the step's input g_n (coefficient a != 0).  Its
// sixteen loads for a cell are issued together, so that the memory latency is
// paid once per cell instead of stalling every store.
// GN: which stages a compiled copy serves.  Per-stage launches take a copy
// without g_n (stage 1) or one that always combines with it (stages 2, 3),
// which issues the loads once its last population's fluxes are in LDS, to
// overlap the last accumulation.  The persistent kernel, which runs all three
// stages with its registers at their limit, tests a at run time and loads
// each value where it is stored: measured in its C4 ensemble, that ran 8 %
// faster than the batch at the start of the epilogue or in the last
// accumulation.
enum { GN_NONE = 0, GN_LOAD = 1, GN_RUNTIME = 2 };
template <class St, int NQ, int GN>
__device__ __forceinline__ void load_gn(const RunDesc& D, const ConstsT<typename St::T>& C, int cs, int cq,
                                        typename St::T (&gnv)[NQ * NQ]) {
    constexpr int NK = NQ * NQ;
    constexpr int B = St::B;
    if (GN == GN_LOAD) {
        const uint32_t planeB = (uint32_t)D.nt * (uint32_t)D.np * B;
        const rsrc_t rgn = make_rsrc(D.gn, NK * planeB);
        const uint32_t cvo = ((uint32_t)cs * (uint32_t)D.np + (uint32_t)cq) * B;
#pragma unroll
        for (int k = 0; k < NK; ++k) gnv[k] = St::bld(rgn, cvo, (uint32_t)k * planeB, (float)C.iscale[k]);
    }
}

template <class St, int NQ, int GN>
__device__ __forceinline__ void stage_epilogue(const RunDesc& D, const ConstsT<typename St::T>& C,
                                               typename St::T (&acc)[NQ * NQ],
                                               const typename St::T (&gk)[NQ * NQ],
                                               typename St::T (&gnv)[NQ * NQ],
                                               typename St::T drho, typename St::T jt,
                                               typename St::T jp, int cs, int cq, uint32_t ctr) {
    // No implicit multiply-add contraction here: every fused operation is
    // written as fma(), so each value rounds the same way in every compiled
    // copy (the compiler's contraction choices follow the block structure,
    // which differs between the per-stage and the persistent kernels).
#pragma clang fp contract(off)
    constexpr int NK = NQ * NQ;
    using T = typename St::T;
    constexpr int B = St::B;
    const int np = D.np;
    const uint32_t planeB = (uint32_t)D.nt * (uint32_t)D.np * B;
    const T dti = uni<T>(D, U_DTI);
    auto vsgn = [](int i) { return 2 * i + 1 < NQ ? -1 : (2 * i + 1 > NQ ? 1 : 0); };
    auto vouter = [](int i) { return i == 0 || i == NQ - 1; };
    // Equilibrium part of BGK from the accumulated moments, eq. (feq_Q=4):
    // f^eq_k = w_k rho (1 + P(xi_k)), xi_k = v_k . u, P(xi) = xi + (xi^2 - u^2)/2
    // + xi (xi^2 - 3 u^2)/6 (Q = 3 drops the cubic term, eq. (feq_Q=3)), with
    // the coefficients 1, 1, 3 taken from the rule's moments (eq_e1, eq_hb,
    // eq_g6: exact mass and momentum on the FP32 rule).  The mirrored
    // population NK-1-k has -xi and the same weight, so each pair shares the
    // even part of P and flips the sign of its odd part, which is formed as
    // xi + xi (...) so that no rounding scales the linear term.
    if constexpr (sizeof(T) != 8) {
        // moments of the kept inputs from the row sums S_kt and column sums P_kp:
        // the nodes are -v_o, -v_i, v_i, v_o (Q = 3: -v_o, 0, v_o)
        T S[NQ], P[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            S[i] = gk[i * NQ];
            P[i] = gk[i];
#pragma unroll
            for (int j = 1; j < NQ; ++j) {
                S[i] += gk[i * NQ + j];
                P[i] += gk[j * NQ + i];
            }
        }
        drho = S[0];
#pragma unroll
        for (int i = 1; i < NQ; ++i) drho += S[i];
        jt = C.v[NQ - 1] * (S[NQ - 1] - S[0]);
        jp = C.v[NQ - 1] * (P[NQ - 1] - P[0]);
        if constexpr (NQ == 4) {
            jt = fma(C.v[2], S[2] - S[1], jt);
            jp = fma(C.v[2], P[2] - P[1], jp);
        }
    }
    const T rho0 = uni<T>(D, U_RHO0);
    const T rho = rho0 + drho;
    const T irho = rcp_nr(rho);
    const T ut = jt * irho, up = jp * irho;
    const T u2 = fma(up, up, ut * ut);
    const T ev0 = C.eq_hb * u2;
    const T cu = fma(-C.eq_g6, u2, C.eq_e1);
    // v_o u and v_i u (theta and phi components); the inner node is 0 for Q = 3
    const T ato = C.v[NQ - 1] * ut, apo = C.v[NQ - 1] * up;
    const T ati = NQ == 4 ? C.v[NQ / 2] * ut : T(0), api = NQ == 4 ? C.v[NQ / 2] * up : T(0);
    auto xi_of = [&](int k) {
        const int kt = k / NQ, kp = k % NQ;
        const T a = vouter(kt) ? ato : ati, b = vouter(kp) ? apo : api;
        return (vsgn(kt) < 0 ? -a : a) + (vsgn(kp) < 0 ? -b : b);
    };
    const T ca = uni<T>(D, U_A), cb = uni<T>(D, U_B);
    const rsrc_t rout = make_rsrc(D.out, NK * planeB);
    const uint32_t cvo = ((uint32_t)cs * (uint32_t)np + (uint32_t)cq) * B;
    // float kernels.  A reduced-precision store adds, every stage, nearly the
    // same increment to nearly the same value: rounding to nearest then makes
    // nearly the same error every step, and those errors add up coherently
    // (linear instead of square-root growth in the number of steps).  Two
    // measures keep the error at rounding level:
    //  - the register sums hold only the increment dt L (the stage input g of
    //    the cell is kept aside in registers), so the arithmetic rounds at the
    //    scale of the increment, and g + increment is rounded once;
    //  - that one rounding is dithered: a value uniform in [-1/2, 1/2) ulp is
    //    added before rounding to nearest, which makes the rounding unbiased
    //    (stochastic rounding).  The dither of population k is h + k c mod
    //    2^32 (c = 2^32 (sqrt5 - 1)/2, a Weyl step), where h is a 32-bit hash
    //    (the "lowbias32" xorshift-multiply mixer) of the cell index, the
    //    step counter and the stage.  A dither shared by all cells would
    //    resonate with cells whose per-step increment matches its own step.
    //    It depends on the step count only, so batched, single and
    //    graph-replayed steps give identical bits.
    uint32_t hsh = 0;
    if constexpr (sizeof(T) != 8) {
        hsh = ((uint32_t)cs * (uint32_t)np + (uint32_t)cq) ^ (ctr * 0x9E3779B9u + D.seq * 0x85EBCA6Bu);
        hsh ^= hsh >> 16; hsh *= 0x7feb352du;
        hsh ^= hsh >> 15; hsh *= 0x846ca68bu;
        hsh ^= hsh >> 16;
    }
    {
        // combine with g_n: always (GN_LOAD, from gnv), never (GN_NONE) or
        // where a != 0 (GN_RUNTIME, loaded here)
        const rsrc_t rgn = make_rsrc(D.gn, NK * planeB);
        auto gn_of = [&](int k) -> T {
            if constexpr (GN == GN_LOAD) return gnv[k];
            else return St::bld(rgn, cvo, (uint32_t)k * planeB, (float)C.iscale[k]);
        };
        // store population k, whose equilibrium deviation is w_k (drho + rho P)
        auto finish = [&](int k, T t) {
            if constexpr (sizeof(T) == 8) {
                // FP64: y = g + dt L was accumulated directly; out = a g_n + b y
                const T y = fma(dti * C.wk[k], t, acc[k]);
                T o = cb * y;
                if (GN == GN_LOAD || (GN == GN_RUNTIME && ca != T(0))) o = fma(ca, gn_of(k), o);
                St::bst(rout, cvo, (uint32_t)k * planeB, o, (float)C.scale[k]);
            } else {
                const T g = gk[k];
                // out = a g_n + b (g + inc) = g + [a (g_n - g) + b inc]; the float
                // kernels' row factors, rest table and dt/tau come multiplied by b
                T d = fma(dti, fma(C.wk[k], t, -g), acc[k]);
                if (GN == GN_LOAD || (GN == GN_RUNTIME && ca != T(0))) d = fma(ca, gn_of(k) - g, d);
                const float x = (float)(int32_t)(hsh + (uint32_t)k * 0x9E3779B9u);
                St::bst_dither(rout, cvo, (uint32_t)k * planeB, g, d, x, (float)C.scale[k]);
            }
        };
        // drho + rho P for each population and its mirror, stored pair by pair
#pragma unroll
        for (int k = 0; 2 * k < NK - 1; ++k) {
            const T xi = xi_of(k);
            const T x2 = xi * xi;
            const T base = fma(rho, fma(T(0.5), x2, ev0), drho);
            T od;
            if constexpr (NQ == 4) od = fma(xi, fma(x2, T(1.0 / 6.0), cu), xi);
            else od = fma(xi, C.eq_e1, xi);
            finish(k, fma(rho, od, base));
            finish(NK - 1 - k, fma(-rho, od, base));
        }
        if constexpr (NK & 1) finish(NK / 2, fma(rho, ev0, drho));     // xi = 0
    }
}

// One tile of one run at one RK stage: tile t of the run described by D, whose
// reduced-precision stores take the dither phase of step ctr.  Every thread of
// the workgroup calls it; it ends after its last barrier (threads without a
// cell return before the epilogue).
template <class St, class Tl, int VAR, int NQ, int GN>
__device__ __forceinline__ void stage_tile(const StageArgs& A, const RunDesc& D, int t, uint32_t ctr) {
    constexpr bool GEN = VAR != VAR_WENO, UPW = VAR == VAR_UPWIND;
    constexpr int NK = NQ * NQ;
    constexpr int TS = Tl::TS, TQ = Tl::TQ, LR = Tl::LR;
    constexpr int NLOAD = Tl::NLOAD, NFT = Tl::NFT, NFP = Tl::NFP;
    using T = typename St::T;
    constexpr int B = St::B;
    using SL = SlotLayout<Tl, (int)sizeof(T)>;
    // FP64 fills its ring with direct-to-LDS loads (no registers hold the
    // populations in flight, no LDS writes place them): each slot is the full
    // LR x LC rectangle, row-major (SlotLayout's 8-byte form), in an LDS
    // object of its own; an interior tile takes it as chunks of two
    // neighbouring values, one 16-byte load per thread landing at byte 16 tid
    // of the slot, a tile with pole rows or a phi wrap in its halo (where
    // neighbouring halo values need not be neighbours in memory) dword by
    // dword, at offsets each thread formed for its dwords at the tile's start.
    // The theta flux function sin(theta) g is formed at the read from a table
    // of the tile's rows.  The float formats interleave the
    // three ring slots element by element (element i of slot b at 3 i + b): a
    // thread's stencil reads in any slot then sit at small constant offsets
    // from one base address, so no per-slot address arithmetic; they keep
    // sin(theta) g in a second ring.
    constexpr bool DMA = sizeof(T) == 8;
    constexpr int LC = Tl::LC, LT = Tl::LT, NCH = LT / 2;
    static_assert(!DMA || (LC % 2 == 0 && NCH <= NTHR && (LT * sizeof(T)) % 16 == 0), "FP64 ring slots");
    // (FP64: three LDS objects, so that the compiler's bookkeeping of the
    // loads in flight into one slot does not hold up the reads of another)
    __shared__ T tile[DMA ? LT : 3 * SL::SIZE];          // g of one population, cross-shaped halo
    __shared__ T tile1[DMA ? LT : 1];
    __shared__ T tile2[DMA ? LT : 1];
    auto slot_base = [&](int b) -> T* { return b == 0 ? tile : (b == 1 ? tile1 : tile2); };
    __shared__ T tileh[DMA ? 1 : 3 * SL::SIZE];          // sin(theta_j) g_j: theta flux function without its speed
    __shared__ T ssin[DMA ? LR : 1];                     // sin(theta) of the tile's rows (FP64)
    // FP64 on a tile with pole rows or a phi wrap: the byte offset of each
    // dword of a slot (population 0, or NK - 1 on a pole row, whose offset is
    // the only odd one: +1 marks the mirror), written and read by the thread
    // that loads that dword
    __shared__ uint32_t dtab[DMA ? 2 * LT : 1];
    auto slot = [&](int b, int a) -> const T& { return DMA ? slot_base(b)[a] : tile[3 * a + b]; };
    __shared__ T fth[2][NFT];
    __shared__ T fph[2][NFP + 1];              // faces with phi index < TQ row-major, then the TS right faces

    const ConstsT<T>& C = consts_of<T>(A);
    const int tid = threadIdx.x;
    const int nt = D.nt, np = D.np;
    const int tq = (np + TQ - 1) / TQ;
    const int s0 = (t / tq) * TS, q0 = (t % tq) * TQ;
    const uint32_t plane = (uint32_t)nt * (uint32_t)np;
    const uint32_t planeB = plane * B;
    const int half = np > 1 ? np / 2 : 0;
    const rsrc_t rin = make_rsrc(D.gin, NK * planeB);

    // ---- load descriptors.  The byte offset of population k at tile position
    // (r, c) is (k*planeB ^ m) + a: m = 0 for interior rows, m = ~0 for pole
    // ghost rows, which then read population 15 - k.
    // a tile whose halo lies inside the grid (no pole rows, no phi wrap): the
    // descriptors need no folding (uniform per workgroup)
    const bool inner = s0 >= NGH && s0 + TS + NGH <= nt && q0 >= NGH && q0 + TQ + NGH <= np;
    auto locate = [&](int r, int c, uint32_t& a, uint32_t& m) {
        int ss = s0 - NGH + r, qq = q0 - NGH + c;
        bool mir = false;
        if (!inner) {
            // column q0 - 3 + c lies in [-3, np + TQ + 2]: one fold suffices when np >= TQ + 3
            qq = np >= TQ + NGH ? wrap1(qq, np) : wrap(qq, np);
            if (ss < 0) {                   // north pole: row -m <- row m-1 at phi + pi, v -> -v
                ss = -1 - ss;
                mir = true;
                qq = wrap1(qq + half, np);
            } else if (ss >= nt) {          // south pole: row nt-1+m <- row nt-m
                ss = 2 * nt - 1 - ss;
                mir = true;
                qq = wrap1(qq + half, np);
            }
            ss = ss < 0 ? 0 : (ss >= nt ? nt - 1 : ss);   // rows no valid cell reads
        }
        a = (uint32_t)(ss * np + qq) * B + (mir ? (uint32_t)(NK - 1) * planeB + 1u : 0u);
        m = mir ? ~0u : 0u;
    };
    // float formats: two cross-shaped positions per thread; FP64 on an
    // interior tile: chunk tid (row tid / (LC / 2), columns 2 (tid % (LC / 2))
    // and the next)
    uint32_t la[2] = {0u, 0u}, lm[2] = {0u, 0u};
    int ldst[2] = {0, 0};
    T lsin[2] = {T(0), T(0)};
    if constexpr (DMA) {
        if (inner) {
            if (tid < NCH) locate(tid / (LC / 2), 2 * (tid % (LC / 2)), la[0], lm[0]);
        } else {
#pragma unroll
            for (int i = 0; i < (2 * LT + NTHR - 1) / NTHR; ++i) {
                const int d = NTHR * i + tid;
                if (d < 2 * LT) {
                    uint32_t a, m;
                    locate((d >> 1) / LC, (d >> 1) % LC, a, m);
                    dtab[d] = a + (uint32_t)(d & 1) * 4u;
                }
            }
        }
        if (tid < LR) {
            const int js = s0 + tid;                  // sin table index of row s0 - 3 + tid
            ssin[tid] = D.rows.sinv[js < nt + 2 * NGH ? js : nt + 2 * NGH - 1];
        }
    } else {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            int idx = tid + NTHR * j;
            const bool used = idx < NLOAD;
            if (!used) idx = 0;
            int r, c;
            if (idx < LR * TQ) {
                r = idx / TQ;
                c = idx % TQ + NGH;
            } else {
                const int e = idx - LR * TQ, e2 = e % (TS * NGH);
                r = e2 / NGH + NGH;
                c = (e < TS * NGH) ? e2 % NGH : TQ + NGH + e2 % NGH;
            }
            ldst[j] = used ? SL::at(r, c) : SL::DUMMY;
            locate(r, c, la[j], lm[j]);
            const int js = s0 + r;                    // sin table index of row s0 - 3 + r
            lsin[j] = T(D.rows.sinv[js < nt + 2 * NGH ? js : nt + 2 * NGH - 1]);
        }
    }
    // FP64: population k into ring slot b straight from memory (lane i of a
    // wave writes bytes size i .. size (i + 1) - 1 past the wave's base)
    using lds_ptr = __attribute__((address_space(3))) void*;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    auto dma = [&](int k, int b) {
        if constexpr (DMA) {
            const uint32_t kb = (uint32_t)k * planeB;
            if (inner) {
                if (tid < NCH)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, (lds_ptr)(slot_base(b) + 2 * 64 * wv), 16,
                                                             la[0], kb, 0, 0);
            } else {
#pragma unroll
                for (int i = 0; i < (2 * LT + NTHR - 1) / NTHR; ++i) {
                    const int d = NTHR * i + tid;            // dword d of the slot
                    if (d < 2 * LT) {
                        const uint32_t a = dtab[d], m = 0u - (a & 1u);
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(
                            rin, (lds_ptr)((char*)slot_base(b) + 4 * (NTHR * i + 64 * wv)), 4, (kb ^ m) + a, 0,
                            0, 0);
                    }
                }
            }
        }
    };
    auto gload = [&](int k, int j) -> T {
        return St::bld(rin, (((uint32_t)k * planeB) ^ lm[j]) + la[j], 0, (float)C.iscale[k]);
    };
    // the velocity nodes are symmetric: population (kt, kp) moves with theta
    // speed sgn(kt) v_o or sgn(kt) v_i (outer or inner node; Q = 3: v_o or 0)
    auto vsgn = [](int i) { return 2 * i + 1 < NQ ? -1 : (2 * i + 1 > NQ ? 1 : 0); };
    auto vouter = [](int i) { return i == 0 || i == NQ - 1; };
    auto lstore = [&](int k, int buf, T v0, T v1) {
        tile[3 * ldst[0] + buf] = v0;
        tile[3 * ldst[1] + buf] = v1;
        if (vsgn(k / NQ) != 0) {              // theta flux function without its speed
            tileh[3 * ldst[0] + buf] = lsin[0] * v0;
            tileh[3 * ldst[1] + buf] = lsin[1] * v1;
        }
    };

    // ---- theta interface of this thread: between tile rows ti-1 and ti, column tc
    const int ti = tid / TQ, tc = tid % TQ;
    const int tbase0 = SL::at(ti, tc + NGH);             // LDS rows ti, ti+2, ti+4
    const int tbase1 = SL::at(ti + 1, tc + NGH);         // LDS rows ti+1, ti+3, ti+5
    const int ig = s0 + ti < nt ? s0 + ti : nt;          // global interface index
    const int scheme = UPW ? D.scheme : (int)VLBM_ADV_WENO5;
    // ---- phi interface of this thread: the left face of its cell for the 240
    // cell threads, the right faces of column 15 for threads 240..254
    const bool phas = tid < NFP;
    // (the idle threads past NFP evaluate a copy of the last right face: every
    // thread runs the same code and only the faces' owners store)
    const int pr = tid < TS * TQ ? tid / TQ : min(tid - TS * TQ, TS - 1);
    const int pj = tid < TS * TQ ? tid % TQ : TQ;
    const int pbase = SL::at(pr + NGH, pj);              // LDS columns pj .. pj+5
    const int pslot = pj < TQ ? pr * TQ + pj : TS * TQ + pr;
    // ---- cell of this thread
    const int cr = tid / TQ, cc = tid % TQ;
    const int cs = s0 + cr, cq = q0 + cc;
    const bool cell = tid < TS * TQ;
    const bool valid = cell && cs < nt && cq < np;
    const int csc = cs < nt ? cs : nt - 1;
    const int rslot = cc + 1 < TQ ? cr * TQ + cc + 1 : TS * TQ + cr;   // right face of the cell
    // per-row factors of the thread's theta interface (fk) and cell (rk).  FP64
    // keeps its tile's rows in LDS and reads each factor where it is used:
    // held in registers they would cost a wave per SIMD (18 registers), and
    // the FP64 kernel's throughput follows its occupancy
    // (only the fields the variant uses: 4 or 5 face values, 5 cell values
    // per row, which keeps five workgroups' LDS within a CU)
    constexpr bool ROWS_LDS = sizeof(T) == 8;
    constexpr int NFK = GEN ? 5 : 4, NRK = 5;
    __shared__ T sfk[ROWS_LDS ? (TS + 1) * NFK : 1];
    __shared__ T srk[ROWS_LDS ? TS * NRK : 1];
    FaceRowK<T> fkr{};
    CellRowK<T> rkr{};
    if constexpr (ROWS_LDS) {
        if (tid < TS + 1) {
            const FaceRowK<T> f = static_cast<const FaceRowK<T>*>(D.facek)[s0 + tid < nt ? s0 + tid : nt];
            T* o = sfk + tid * NFK;
            o[0] = f.cp1; o[1] = f.cp3; o[2] = f.cm1; o[3] = f.cm3;
            if constexpr (GEN) o[4] = f.sI;
        } else if (tid >= 64 && tid < 64 + TS) {
            const CellRowK<T> c = static_cast<const CellRowK<T>*>(D.rowk)[s0 + tid - 64 < nt ? s0 + tid - 64 : nt - 1];
            T* o = srk + (tid - 64) * NRK;
            o[0] = c.th_o; o[1] = c.th_i; o[2] = c.ph_o; o[3] = c.ph_i; o[4] = c.dtcot;
        }
    } else {
        fkr = static_cast<const FaceRowK<T>*>(D.facek)[ig];
        rkr = static_cast<const CellRowK<T>*>(D.rowk)[csc];
    }
    // face factor i of the thread's theta interface: cp1, cp3, cm1, cm3, sI
    auto FK = [&](int i) -> T {
        if constexpr (ROWS_LDS) return sfk[ti * NFK + i];
        else return i == 0 ? fkr.cp1 : i == 1 ? fkr.cp3 : i == 2 ? fkr.cm1 : i == 3 ? fkr.cm3 : fkr.sI;
    };
    // cell factor i of the thread's row: th_o, th_i, ph_o, ph_i, dtcot
    auto RK = [&](int i) -> T {
        if constexpr (ROWS_LDS) return srk[cr * NRK + i];
        else return i == 0 ? rkr.th_o : i == 1 ? rkr.th_i : i == 2 ? rkr.ph_o : i == 3 ? rkr.ph_i : rkr.dtcot;
    };
    const T epsk = uni<T>(D, U_EPSK);
    const void* rest_t = sizeof(T) == 8 ? static_cast<const void*>(D.rows.rest)
                                        : static_cast<const void*>(D.rest_f);
    const rsrc_t rrest = make_rsrc(rest_t, (uint32_t)(NK * nt * sizeof(T)));
    const uint32_t rvo = (uint32_t)csc * (uint32_t)sizeof(T);

    // the sums start from the rest state's dt L of the cell's row
    T acc[NK];
    T gk[NK];   // the cell's stage input, kept for the float epilogue
    T gnv[NK];  // the step's input g_n (stages 2 and 3)
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        acc[k] = St::rload(rrest, rvo, (uint32_t)(k * nt) * (uint32_t)sizeof(T));
        gk[k] = T(0);
    }
    T drho = T(0), jt = T(0), jp = T(0);
    // the loop's uniform constants, read once into scalar registers so that the
    // population loop issues no scalar loads (whose waits would also wait for
    // the outstanding LDS reads).  The force uses the kernels K^H, K~^H, not
    // their products with the node speeds.  FP64 keeps only the rows of the
    // first (Q+1)/2 nodes, which fit the scalar registers: the nodes are
    // symmetric (v_{Q-1-i} = -v_i, H_n(-x) = (-1)^n H_n(x)), so
    // K^H[Q-1-i][Q-1-j] = -K^H[i][j], K~^H[Q-1-i][Q-1-j] = K~^H[i][j] and
    // w_k depends on the folded node indices only.
    constexpr bool FOLD = sizeof(T) == 8;
    constexpr int NH = (NQ + 1) / 2;
    constexpr int NKR = FOLD ? NH * NQ : NK, NVR = FOLD ? NH : NQ, NWR = FOLD ? NH * NH : NK;
    T CK[NKR], CKt[NKR], Cwr[NWR], Cv[NVR], Cnv2[NVR];
#pragma unroll
    for (int i = 0; i < NKR; ++i) { CK[i] = C.K[i]; CKt[i] = C.Kt[i]; }
#pragma unroll
    for (int i = 0; i < NWR; ++i) Cwr[i] = FOLD ? C.wr[(i / NH) * NQ + i % NH] : C.wr[i];
#pragma unroll
    for (int i = 0; i < NVR; ++i) { Cv[i] = C.v[i]; Cnv2[i] = C.nv2[i]; }
    auto mir = [](int i) { return FOLD && 2 * i >= NQ; };
    auto fold = [&](int i) { return mir(i) ? NQ - 1 - i : i; };
    auto kK = [&](int i, int j) { return mir(i) ? -CK[fold(i) * NQ + NQ - 1 - j] : CK[i * NQ + j]; };
    auto kKt = [&](int i, int j) { return mir(i) ? CKt[fold(i) * NQ + NQ - 1 - j] : CKt[i * NQ + j]; };
    auto nodev = [&](int i) { return mir(i) ? -Cv[fold(i)] : Cv[i]; };
    auto nodenv2 = [&](int i) { return Cnv2[fold(i)]; };
    auto wrk = [&](int kt, int kp) { return FOLD ? Cwr[fold(kt) * NH + fold(kp)] : Cwr[kt * NQ + kp]; };

    // Populations are taken in the order ord(i) (D2Q16: the sign-sharing
    // rounds of stage_tile_rounds, so that both kernels accumulate every cell
    // in the same order and give the same bits).  Ring of three LDS slots:
    // the i-th population lives in slot i % 3 and is written to LDS at the end
    // of iteration i - 2, when the slot of iteration i - 3 has been read for
    // the last time.  Its global loads are issued PF iterations ahead, at the
    // start of iteration i - PF, into the register pair nx[i % 2]: the float
    // kernels (7 waves) give them one iteration to arrive.  FP64 loads the
    // i-th population straight into its slot after the barrier of iteration
    // i - 3, the last that reads that slot; it must be in LDS for every wave
    // after the barrier of iteration i - 1, two iterations later.
    auto ord = [](int i) { return NQ == 4 ? ROUND_ORDER[i] : i; };
    constexpr int PF = 2;
    T nx[2][2];
    if constexpr (DMA) {
        dma(ord(0), 0);
        dma(ord(1), 1);
        dma(ord(2), 2);
        __builtin_amdgcn_s_waitcnt(0x0f70);           // vmcnt 0 (the barrier's release needs it too)
    } else {
        const T a0 = gload(ord(0), 0), a1 = gload(ord(0), 1), b0 = gload(ord(1), 0), b1 = gload(ord(1), 1);
        lstore(ord(0), 0, a0, a1);
        lstore(ord(1), 1, b0, b1);
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < NK; ++i) {
        const int k = ord(i);
        const int kt = k / NQ, kp = k % NQ;
        const int tb = i % 3, fb = i & 1;
        // theta and phi speeds of this population (zero: no flux in that direction)
        const int st = vsgn(kt), sp = vsgn(kp);
        T gself = T(0), Ftself = T(0), Flself = T(0);
        // global loads of the population PF iterations ahead (float formats)
        if (!DMA && i + PF < NK) {
            nx[(i + PF) & 1][0] = gload(ord(i + PF), 0);
            nx[(i + PF) & 1][1] = gload(ord(i + PF), 1);
        }
        // theta flux of sin(theta_j) g_j (the speed multiplies the difference)
        if (st != 0) {
            T g[6], h[6];
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                const int a = (m & 1 ? tbase1 : tbase0) + (m >> 1) * SL::RS2;
                g[m] = slot(tb, a);
                if constexpr (DMA) {
                    h[m] = ssin[ti + m] * g[m];
                    // a rounded product, as the float formats' second ring holds:
                    // kept out of multiply-add contraction with the differences
                    // the candidates take of it
                    asm("" : "+v"(h[m]));
                } else {
                    h[m] = tileh[3 * a + tb];
                }
            }
            gself = g[3];                                // this thread's cell (row ti, column tc)
            T F;
            if constexpr (!UPW) {
                if (st > 0)
                    F = weno5x6<T, true>(h[0], h[1], h[2], h[3], h[4], g[0], g[1], g[2], g[3], g[4],
                                         epsk, wrk(kt, kp), FK(0), FK(1));
                else
                    F = weno5x6<T, true>(h[5], h[4], h[3], h[2], h[1], g[5], g[4], g[3], g[2], g[1],
                                         epsk, wrk(kt, kp), FK(2), FK(3));
            } else {
                F = st > 0 ? upwind(scheme, h[1], h[2], h[3]) : upwind(scheme, h[4], h[3], h[2]);
            }
            if constexpr (GEN) F *= FK(4);
            fth[fb][tid] = F;
            Ftself = F;                                  // top face of this thread's cell
        } else {
            gself = slot(tb, tbase1 + SL::RS2);          // LDS row ti+3
        }
        // phi flux of g (the speed multiplies the difference)
        if (sp != 0) {
            T g[6];
#pragma unroll
            for (int m = 0; m < 6; ++m) g[m] = slot(tb, pbase + m);
            T F;
            if constexpr (!UPW) {
                if (sp > 0)
                    F = weno5x6<T, false>(g[0], g[1], g[2], g[3], g[4], g[0], g[1], g[2], g[3], g[4],
                                          epsk, T(0), T(0), T(0));
                else
                    F = weno5x6<T, false>(g[5], g[4], g[3], g[2], g[1], g[5], g[4], g[3], g[2], g[1],
                                          epsk, T(0), T(0), T(0));
            } else {
                F = sp > 0 ? upwind(scheme, g[1], g[2], g[3]) : upwind(scheme, g[4], g[3], g[2]);
            }
            Flself = F;                                  // left face of this thread's cell
            if (phas) fph[fb][pslot] = F;
        }
        if constexpr (DMA) {
            // a plain barrier (a __syncthreads() would wait for all of the
            // wave's direct-to-LDS loads): this wave's LDS reads and face writes
            // done (lgkmcnt 0), and of its direct loads only population i + 2's
            // still outstanding (an interior tile issues one per population;
            // a border tile waits for all); the empty asm statements keep the
            // compiler from moving memory accesses across
            asm volatile("" ::: "memory");
            if (inner && i + 2 < NK) __builtin_amdgcn_s_waitcnt(0x0071);   // vmcnt 1, lgkmcnt 0
            else __builtin_amdgcn_s_waitcnt(0x0070);                       // vmcnt 0, lgkmcnt 0
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
        } else {
            __syncthreads();
        }
        // FP64: population i + 3 into the slot this iteration has finished reading
        if (DMA && i + 3 < NK) dma(ord(i + 3), tb);
        if (GN == GN_LOAD && i == NK - 1 && valid) load_gn<St, NQ, GN>(D, C, cs, cq, gnv);
        if (cell) {
            const T gc = gself;
            // FP64 folds the BGK loss -g/tau in here; the float kernels form the
            // whole collision term at the end (see the epilogue)
            T a = acc[k];
            if constexpr (sizeof(T) == 8) a = fma(uni<T>(D, U_OMDTI), gc, a);
            if (st != 0) {                               // - v_theta dt/(R sin th dth) (F_b - F_t)
                const T Fb = fth[fb][(cr + 1) * TQ + cc];
                const T f = RK(vouter(kt) ? 0 : 1);
                a = fma(st > 0 ? -f : f, Fb - Ftself, a);
            }
            if (sp != 0) {                               // - v_phi dt/(R sin th dph) (F_r - F_l)
                const T Fr = fph[fb][rslot];
                const T f = RK(vouter(kp) ? 2 : 3);
                a = fma(sp > 0 ? -f : f, Fr - Flself, a);
            }
            acc[k] = a;
            // rank-1 force updates: -v_kp^2 K[b][kt] and v_kt K~[b][kp] times
            // dt cot(theta)/R g, applied as two scalings of tg
            const T tg = RK(4) * gc;
            const T ta = nodenv2(kp) * tg, tb = nodev(kt) * tg;
#pragma unroll
            for (int b = 0; b < NQ; ++b) {
                acc[b * NQ + kp] = fma(kK(b, kt), ta, acc[b * NQ + kp]);
                acc[kt * NQ + b] = fma(kKt(b, kp), tb, acc[kt * NQ + b]);
            }
            if constexpr (sizeof(T) != 8) {
                gk[k] = gc;                          // moments from these at the end
            } else {
                drho += gc;
                jt = fma(nodev(kt), gc, jt);
                jp = fma(nodev(kp), gc, jp);
            }
        }
        if (!DMA && i + 2 < NK) lstore(ord(i + 2), (i + 2) % 3, nx[i & 1][0], nx[i & 1][1]);
        // keep this population's register arithmetic in place: deferring it past
        // the following barriers would keep every population's inputs live at once
        if constexpr (NK == 16)
            asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]),
                         "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7]), "+v"(acc[8]), "+v"(acc[9]),
                         "+v"(acc[10]), "+v"(acc[11]), "+v"(acc[12]), "+v"(acc[13]), "+v"(acc[14]),
                         "+v"(acc[15]));
        else
            asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]),
                         "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7]), "+v"(acc[8]));
        if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(drho), "+v"(jt), "+v"(jp));
    }

    if (!valid) return;
    stage_epilogue<St, NQ, GN>(D, C, acc, gk, gnv, drho, jt, jp, cs, cq, ctr);
}

// ---------------------------------------------------------------------------
// Fused RK stage in population rounds (D2Q16, WENO-5 standard form or an
// upwind scheme in either theta form, 15 x 16 tiles): the same operator,
// per-face arithmetic and per-cell order of
// accumulation as stage_tile, hence the same bits, with less LDS traffic and
// a quarter of its barriers.
//
// The populations are taken four at a time in the rounds of ROUND_ORDER, whose
// members share the signs of both speed components, so every flux of a round
// is upwinded the same way.  A round's four tiles sit in LDS together.  Wave
// w computes the theta fluxes of interface rows 4w .. 4w+3 of
// all four populations (lane = population x column), walking down its column:
// the eight stencil rows are read once for four interfaces, sin(theta) of a row
// is the same for the whole wave, and the differences the interfaces share are
// formed once.  The phi fluxes go the same way along the rows (lane =
// population x row; interfaces 4w .. 4w+3, wave 3 also the tile's right edge).
// Then the 240 cell threads read the four faces of each of the round's
// populations and accumulate as in stage_tile.  The loads of later rounds are
// in flight meanwhile (FP32: straight into a second tile set; FP16: in
// registers, written to LDS once the fluxes have been read): two barriers per
// round, eight per stage.
template <class T>
__device__ __forceinline__ T scalar_load(const T* p, int i) {
    // the row tables are written before any launch and only read by kernels:
    // read through the constant address space, an index that is uniform over
    // the workgroup then gives a scalar load
    return ((const __attribute__((address_space(4))) T*)p)[i];
}

template <class St, int VAR, bool LDSDMA, int GN>
__device__ __forceinline__ void stage_tile_rounds(const StageArgs& A, const RunDesc& D, int t, uint32_t ctr) {
    using Tl = Tile15x16;
    constexpr int NQ = 4, NK = 16;
    constexpr int TS = Tl::TS, TQ = Tl::TQ, LR = Tl::LR, NLOAD = Tl::NLOAD;
    using T = typename St::T;
    constexpr int B = St::B;
    // FP32 on one large run (a stored value is the arithmetic value) fills
    // its tiles with direct-to-LDS loads, so no registers hold the coming
    // rounds in flight:
    // the tile is the full LR x LC rectangle, row-major with pitch LC = 22,
    // taken dword by dword (lane i of a wave writes dword i past the wave's
    // base), each dword at its own folded address, so pole rows and the phi
    // wrap need no special case.  Two tile sets alternate between rounds, so
    // the loads of round r + 2 are issued while round r + 1 is computed.  The
    // 16 rows of a phi read (22 dwords apart) fall on distinct banks; the
    // populations' tiles are 464 dwords apart (16 modulo 64 banks), so the
    // four 16-lane groups of a theta read take disjoint banks.  FP16
    // (converted and scaled on the way in), batches of runs and small runs
    // keep one cross-shaped tile set of pitch 23 filled through registers;
    // the unused last column of row 0 takes the writes of unused load slots.
    constexpr bool DMA = LDSDMA;
    static_assert(!DMA || (B == (int)sizeof(T) && sizeof(T) == 4), "direct-to-LDS loads copy FP32 values");
    constexpr int LC = TQ + 2 * NGH;
    constexpr int PITCH = DMA ? LC : 23, PSZ = DMA ? 464 : LR * PITCH, DUMMY = PITCH - 1;
    constexpr int NDW = LR * LC, NSL = (NDW + NTHR - 1) / NTHR;   // dwords of a DMA tile, per thread
    static_assert(!DMA || (LR * LC <= PSZ && NSL == 2), "direct-to-LDS tile");
    constexpr int FTP = (TS + 1) * TQ;          // theta faces of a population
    constexpr int FPR = TQ + 1, FPP = TS * FPR;  // phi faces per row, per population
    constexpr int NBUF = DMA ? 2 : 1;            // FP32: rounds alternate between two tile sets
    __shared__ T tile[NBUF * 4 * PSZ];
    __shared__ T fth[4 * FTP];
    __shared__ T fph[4 * FPP];

    const ConstsT<T>& C = consts_of<T>(A);
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);     // wave of the workgroup
    const int lp = (tid & 63) >> 4, l16 = tid & 15;
    const int nt = D.nt, np = D.np;
    const int tq = (np + TQ - 1) / TQ;
    const int s0 = (t / tq) * TS, q0 = (t % tq) * TQ;
    const uint32_t planeB = (uint32_t)nt * (uint32_t)np * B;
    const int half = np > 1 ? np / 2 : 0;
    const rsrc_t rin = make_rsrc(D.gin, NK * planeB);

    // ---- load descriptors (as stage_tile): two positions per thread (FP32:
    // dwords tid and tid + 256 of the rectangle, FP16: cross-shaped
    // positions); population k at byte offset (k planeB ^ m) + a
    uint32_t la[2], lm[2];
    int ldst[2];
    const bool inner = s0 >= NGH && s0 + TS + NGH <= nt && q0 >= NGH && q0 + TQ + NGH <= np;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        int idx = tid + NTHR * j;
        const bool used = idx < (DMA ? NDW : NLOAD);
        if (!used) idx = 0;
        int r, c;
        if constexpr (DMA) {
            r = idx / LC;
            c = idx % LC;
        } else if (idx < LR * TQ) {
            r = idx / TQ;
            c = idx % TQ + NGH;
        } else {
            const int e = idx - LR * TQ, e2 = e % (TS * NGH);
            r = e2 / NGH + NGH;
            c = (e < TS * NGH) ? e2 % NGH : TQ + NGH + e2 % NGH;
        }
        int ss = s0 - NGH + r, qq = q0 - NGH + c;
        bool mir = false;
        if (!inner) {
            qq = np >= TQ + NGH ? wrap1(qq, np) : wrap(qq, np);
            if (ss < 0) {
                ss = -1 - ss;
                mir = true;
                qq = wrap1(qq + half, np);
            } else if (ss >= nt) {
                ss = 2 * nt - 1 - ss;
                mir = true;
                qq = wrap1(qq + half, np);
            }
            ss = ss < 0 ? 0 : (ss >= nt ? nt - 1 : ss);
        }
        ldst[j] = used ? r * PITCH + c : DUMMY;
        la[j] = (uint32_t)(ss * np + qq) * B + (mir ? (uint32_t)(NK - 1) * planeB + 1u : 0u);
        lm[j] = mir ? ~0u : 0u;
    }
    auto gload = [&](int k, int j) -> T {
        return St::bld(rin, (((uint32_t)k * planeB) ^ lm[j]) + la[j], 0, (float)C.iscale[k]);
    };
    auto vouter = [](int i) { return i == 0 || i == NQ - 1; };

    // ---- this thread's cell
    const int cr = tid / TQ, cc = tid % TQ;
    const int cs = s0 + cr, cq = q0 + cc;
    const bool cell = tid < TS * TQ;
    const bool valid = cell && cs < nt && cq < np;
    const int csc = cs < nt ? cs : nt - 1;
    const CellRowK<T> rkr = static_cast<const CellRowK<T>*>(D.rowk)[csc];
    const T epsk = uni<T>(D, U_EPSK);
    const int scheme = D.scheme;                 // U1 / U2 / U3 (upwind variant)
    const void* rest_t = sizeof(T) == 8 ? static_cast<const void*>(D.rows.rest)
                                        : static_cast<const void*>(D.rest_f);
    const rsrc_t rrest = make_rsrc(rest_t, (uint32_t)(NK * nt * sizeof(T)));
    const uint32_t rvo = (uint32_t)csc * (uint32_t)sizeof(T);
    T acc[NK];
    T gk[NK];
    T gnv[NK];  // the step's input g_n (stages 2 and 3)
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        acc[k] = St::rload(rrest, rvo, (uint32_t)(k * nt) * (uint32_t)sizeof(T));
        gk[k] = T(0);
    }
    T drho = T(0), jt = T(0), jp = T(0);
    // rule constants in scalar registers: only the rows of the first two nodes,
    // the others by the node symmetry (exact in both arithmetic types: the FP32
    // nodes are symmetric too), so the values equal stage_tile's
    constexpr bool FOLD = true;
    constexpr int NH = 2;
    constexpr int NKR = FOLD ? NH * NQ : NK, NVR = FOLD ? NH : NQ, NWR = FOLD ? NH * NH : NK;
    T CK[NKR], CKt[NKR], Cwr[NWR], Cv[NVR], Cnv2[NVR];
#pragma unroll
    for (int i = 0; i < NKR; ++i) { CK[i] = C.K[i]; CKt[i] = C.Kt[i]; }
#pragma unroll
    for (int i = 0; i < NWR; ++i) Cwr[i] = FOLD ? C.wr[(i / NH) * NQ + i % NH] : C.wr[i];
#pragma unroll
    for (int i = 0; i < NVR; ++i) { Cv[i] = C.v[i]; Cnv2[i] = C.nv2[i]; }
    auto mir = [](int i) { return FOLD && 2 * i >= NQ; };
    auto fold = [&](int i) { return mir(i) ? NQ - 1 - i : i; };
    auto kK = [&](int i, int j) { return mir(i) ? -CK[fold(i) * NQ + NQ - 1 - j] : CK[i * NQ + j]; };
    auto kKt = [&](int i, int j) { return mir(i) ? CKt[fold(i) * NQ + NQ - 1 - j] : CKt[i * NQ + j]; };
    auto nodev = [&](int i) { return mir(i) ? -Cv[fold(i)] : Cv[i]; };
    auto nodenv2 = [&](int i) { return Cnv2[fold(i)]; };
    auto wrk = [&](int kt, int kp) { return FOLD ? Cwr[fold(kt) * NH + fold(kp)] : Cwr[kt * NQ + kp]; };

    // the loads of round r: population ROUND_ORDER[4 r + p] of both positions
    // (FP32: straight into LDS, at dwords j 256 + 64 w + lane of the tile)
    T nx[4][2];
    auto issue = [&](int r) {
        if constexpr (DMA) {
            // an interior tile passes the population's offset as the scalar
            // offset (no per-load address arithmetic); a tile with pole rows
            // or a phi wrap folds it into each lane's offset
            auto issue_as = [&](auto interior) {
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const uint32_t kb = (uint32_t)ROUND_ORDER[4 * r + p] * planeB;
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        if (NTHR * j + tid < NDW)
                            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                                rin,
                                (__attribute__((address_space(3))) void*)(tile + ((r & 1) * 4 + p) * PSZ + NTHR * j + 64 * w),
                                4, decltype(interior)::value ? la[j] : (kb ^ lm[j]) + la[j],
                                decltype(interior)::value ? kb : 0u, 0, 0);
                }
            };
            if (inner) issue_as(std::true_type{});
            else issue_as(std::false_type{});
        } else {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                nx[p][0] = gload(ROUND_ORDER[4 * r + p], 0);
                nx[p][1] = gload(ROUND_ORDER[4 * r + p], 1);
            }
        }
    };
    auto put = [&]() {
        if constexpr (!DMA) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                tile[p * PSZ + ldst[0]] = nx[p][0];
                tile[p * PSZ + ldst[1]] = nx[p][1];
            }
        }
    };
    // direct-to-LDS loads count in vmcnt, in issue order, eight per round and
    // wave: before the barrier that makes a round's tiles visible, the wave
    // waits until at most the eight of the round after it are outstanding
    // (vmcnt 8 or 0; expcnt, lgkmcnt unchanged)
    auto dma_done = [&](bool newer) {
        if constexpr (DMA) {
            if (newer) __builtin_amdgcn_s_waitcnt(0x0f78);
            else __builtin_amdgcn_s_waitcnt(0x0f70);
        }
    };
    issue(0);
    put();
    issue(1);
    dma_done(true);
    __syncthreads();

    const FaceRowK<T>* fkt = static_cast<const FaceRowK<T>*>(D.facek);
    // sin(theta) of LDS row 4w + m (the theta flux function without its
    // speed), the value of stage_tile's sin table lookup in the arithmetic
    // type (the float formats read a table rounded on the host); uniform per
    // wave, a scalar load where used
    auto sin_row = [&](int m) -> T {
        const int js = s0 + 4 * w + m, j = js < nt + 2 * NGH ? js : nt + 2 * NGH - 1;
        if constexpr (sizeof(T) == 8) return scalar_load(D.rows.sinv, j);
        else return scalar_load(D.sinv_f, j);
    };

#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int st = r < 2 ? -1 : 1;              // sign of v_theta in this round
        const int sp = (r & 1) ? 1 : -1;            // sign of v_phi
        const T* tl = tile + ((DMA ? (r & 1) * 4 : 0) + lp) * PSZ;
        const T* rt = tile + (DMA ? (r & 1) * 4 : 0) * PSZ;         // the round's tiles
        // -- the cell's own values of the round's populations (FP32: after the
        // fluxes; the next round's loads overwrite the tiles after the barrier)
        T gself[4];
        auto read_self = [&]() {
            if (cell) {
#pragma unroll
                for (int p = 0; p < 4; ++p) gself[p] = rt[p * PSZ + (cr + NGH) * PITCH + cc + NGH];
            }
        };
        if constexpr (!DMA) read_self();
        // -- theta fluxes: population lp, column l16, interface rows 4w .. 4w+3
        if constexpr (VAR == VAR_UPWIND) {
            // upwind: the three points a, b, c of the flux at interface 4w+f
            // are rows 4w+f+1 .. 4w+f+3 (positive speed) or 4w+f+4 .. 4w+f+2;
            // the rest state's part is in the rest table (the flux is linear);
            // the interface factor is sin(theta) at the interface in the
            // Komissarov form, 1 otherwise
            T h[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                if (st > 0 ? (m >= 1 && m <= 6) : (m >= 2 && m <= 7)) {
                    const T S = sin_row(m);
                    h[m] = S * tl[(4 * w + m) * PITCH + l16 + NGH];
                    asm("" : "+v"(h[m]));
                } else {
                    h[m] = T(0);
                }
            }
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int ig = s0 + 4 * w + f < nt ? s0 + 4 * w + f : nt;
                T F = st > 0 ? upwind(scheme, h[f + 1], h[f + 2], h[f + 3])
                             : upwind(scheme, h[f + 4], h[f + 3], h[f + 2]);
                F *= scalar_load(&fkt[ig].sI, 0);
                fth[lp * FTP + (4 * w + f) * TQ + l16] = F;
            }
        } else {

            // the rest weight of this lane's population (a select, not a
            // per-lane table lookup)
            auto wr_of = [&](int p) { return wrk(ROUND_ORDER[4 * r + p] / NQ, ROUND_ORDER[4 * r + p] % NQ); };
            const T wr = lp == 0 ? wr_of(0) : lp == 1 ? wr_of(1) : lp == 2 ? wr_of(2) : wr_of(3);
            T g[9], h[9];
#pragma unroll
            for (int m = 0; m < 9; ++m) {
                if (st > 0 ? m < 8 : m > 0) {
                    const T S = sin_row(m);
                    g[m] = tl[(4 * w + m) * PITCH + l16 + NGH];
                    h[m] = S * g[m];
                    // h is a rounded product, as when stage_tile reads it from
                    // LDS: kept out of multiply-add contraction with the
                    // differences the WENO candidates take of it
                    asm("" : "+v"(h[m]));
                } else {
                    g[m] = h[m] = T(0);
                }
            }
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int ig = s0 + 4 * w + f < nt ? s0 + 4 * w + f : nt;
                T F;
                if (st > 0)
                    F = weno5x6<T, true>(h[f], h[f + 1], h[f + 2], h[f + 3], h[f + 4], g[f], g[f + 1],
                                         g[f + 2], g[f + 3], g[f + 4], epsk, wr,
                                         scalar_load(&fkt[ig].cp1, 0), scalar_load(&fkt[ig].cp3, 0));
                else
                    F = weno5x6<T, true>(h[f + 5], h[f + 4], h[f + 3], h[f + 2], h[f + 1], g[f + 5],
                                         g[f + 4], g[f + 3], g[f + 2], g[f + 1], epsk, wr,
                                         scalar_load(&fkt[ig].cm1, 0), scalar_load(&fkt[ig].cm3, 0));
                fth[lp * FTP + (4 * w + f) * TQ + l16] = F;
            }
        }
        // -- phi fluxes: population lp, row l16 (lane 15 repeats row 14 and
        // stores nothing), interfaces 4w .. 4w+3 (wave 3 also interface 16)
        {
            const int pr = l16 < TS ? l16 : TS - 1;
            const T* row = tl + (pr + NGH) * PITCH + 4 * w;
            T g[10];
#pragma unroll
            for (int m = 0; m < 10; ++m) {
                const bool need = VAR == VAR_UPWIND
                                      ? (sp > 0 ? m >= 1 && (m < 7 || (m < 8 && w == 3))
                                                : m >= 2 && (m < 8 || (m < 9 && w == 3)))
                                      : (sp > 0 ? m < 8 || (m < 9 && w == 3) : (m > 0 && (m < 9 || w == 3)));
                g[m] = need ? row[m] : T(0);
            }
            auto face = [&](int f) {
                T F;
                if constexpr (VAR == VAR_UPWIND)
                    F = sp > 0 ? upwind(scheme, g[f + 1], g[f + 2], g[f + 3])
                               : upwind(scheme, g[f + 4], g[f + 3], g[f + 2]);
                else if (sp > 0)
                    F = weno5x6<T, false>(g[f], g[f + 1], g[f + 2], g[f + 3], g[f + 4], g[f], g[f + 1],
                                          g[f + 2], g[f + 3], g[f + 4], epsk, T(0), T(0), T(0));
                else
                    F = weno5x6<T, false>(g[f + 5], g[f + 4], g[f + 3], g[f + 2], g[f + 1], g[f + 5],
                                          g[f + 4], g[f + 3], g[f + 2], g[f + 1], epsk, T(0), T(0), T(0));
                if (l16 < TS) fph[lp * FPP + pr * FPR + 4 * w + f] = F;
            };
#pragma unroll
            for (int f = 0; f < 4; ++f) face(f);
            if (w == 3) face(4);
        }
        if constexpr (DMA) read_self();
        __syncthreads();
        // -- the next round's tile, then its successor's loads (FP32: the loads
        // of the round after next, into the tile set this round has finished)
        if constexpr (DMA) {
            if (r < 2) issue(r + 2);
        } else if (r < 3) {
            put();
            if (r < 2) issue(r + 2);
        }
        if (GN == GN_LOAD && r == 3 && valid) load_gn<St, NQ, GN>(D, C, cs, cq, gnv);
        // -- the cells accumulate the round's populations in order
        if (cell) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int k = ROUND_ORDER[4 * r + p];
                const int kt = k / NQ, kp = k % NQ;
                const T gc = gself[p];
                T a = acc[k];
                if constexpr (sizeof(T) == 8) a = fma(uni<T>(D, U_OMDTI), gc, a);
                {
                    const T Ft = fth[p * FTP + cr * TQ + cc], Fb = fth[p * FTP + (cr + 1) * TQ + cc];
                    const T f = vouter(kt) ? rkr.th_o : rkr.th_i;
                    a = fma(st > 0 ? -f : f, Fb - Ft, a);
                }
                {
                    const T Fl = fph[p * FPP + cr * FPR + cc], Fr = fph[p * FPP + cr * FPR + cc + 1];
                    const T f = vouter(kp) ? rkr.ph_o : rkr.ph_i;
                    a = fma(sp > 0 ? -f : f, Fr - Fl, a);
                }
                acc[k] = a;
                const T tg = rkr.dtcot * gc;
                const T ta = nodenv2(kp) * tg, tb = nodev(kt) * tg;
#pragma unroll
                for (int b = 0; b < NQ; ++b) {
                    acc[b * NQ + kp] = fma(kK(b, kt), ta, acc[b * NQ + kp]);
                    acc[kt * NQ + b] = fma(kKt(b, kp), tb, acc[kt * NQ + b]);
                }
                if constexpr (sizeof(T) != 8) {
                    gk[k] = gc;
                } else {
                    drho += gc;
                    jt = fma(nodev(kt), gc, jt);
                    jp = fma(nodev(kp), gc, jp);
                }
            }
        }
        if (r < 3) {
            dma_done(r < 2);
            __syncthreads();
        }
    }
    if (!valid) return;
    stage_epilogue<St, NQ, GN>(D, C, acc, gk, gnv, drho, jt, jp, cs, cq, ctr);
}

// the run of global tile tg: the largest run with tile_start[run] <= tg
__device__ __forceinline__ int run_of(const StageArgs& A, int tg) {
    int run = 0, hi = A.nruns - 1;
    while (run < hi) {
        const int mid = (run + hi + 1) >> 1;
        if (A.tile_start[mid] <= tg) run = mid;
        else hi = mid - 1;
    }
    return run;
}

// One RK stage over the tiles of up to MAXRUNS runs, one workgroup per tile.
// Workgroups are numbered so that those sharing an XCD (dispatched round-robin
// over the 8 XCDs) take a contiguous range of tiles, keeping halo rows and the
// 64-byte halves of shared cache lines inside one L2.  A single-run launch reads
// its run from the kernel arguments; a batched one looks up the run of its
// tile (uniform per workgroup).  LDSDMA: the rounds kernel's direct-to-LDS
// form (FP32).
template <class St, bool BATCH, class Tl, int VAR, int NQ, bool LDSDMA, int GN>
__global__ __launch_bounds__(NTHR, (launch_min_waves<St, Tl, VAR, NQ, LDSDMA>())) void stage_kernel(StageArgs A) {
    const int nall = A.tile_start[A.nruns];
    const int per = (nall + 7) / 8;
    const int tg = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tg >= nall) return;                    // whole workgroup leaves before any barrier
    const int run = BATCH ? run_of(A, tg) : 0;
    const RunDesc& D = BATCH ? *A.desc[run] : A.run0;
    const uint32_t ctr = sizeof(typename St::T) == 8 ? 0u : *D.ctr;
    if constexpr (uses_rounds<typename St::T, Tl, VAR, NQ>())
        stage_tile_rounds<St, VAR, LDSDMA, GN>(A, D, tg - A.tile_start[run], ctr);
    else
        stage_tile<St, Tl, VAR, NQ, GN>(A, D, tg - A.tile_start[run], ctr);
}

// ---------------------------------------------------------------------------
// Persistent batched stepping: one cooperative launch carries n steps (3n RK
// stages) of up to MAXRUNS runs.  Its workgroups are co-resident; each takes
// the tiles of a stage with the XCD-aware numbering of stage_kernel, strided
// by the grid size (a multiple of 8, so a workgroup stays on its XCD's range),
// and all meet at a grid barrier before the next stage reads the halos.  The tile arithmetic is stage_tile's, so the results equal per-stage
// launches bit for bit.
struct PersistArgs {
    StageArgs A;           // desc[i]: run i's stage-1 descriptor; stages 2 and 3 follow it
    int nsteps;
    uint32_t spin_limit;   // polls of one barrier wait before it gives up
    uint32_t* bar;         // XCDs through the grid barrier, zero at the launch
    uint32_t* err;         // set to 1 when a barrier wait gave up
    uint32_t* xbar;        // [8] arrivals per XCD, zero at the launch
    uint32_t* xreg;        // [8] workgroups per XCD, then [8] the registration barrier's arrivals; zero at the launch
};
constexpr int PERSIST_WORDS = 2 + 8 + 16;
static_assert(sizeof(PersistArgs) <= 4096, "kernel arguments must fit the 4 KiB kernarg segment");

// Bounded wait until *c reaches target (relaxed polls), then one acquire
// fence: later loads see the stores released before the count.  (An acquire
// on every poll would invalidate the XCD's caches under the workgroups still
// computing.)  After spin_limit polls, or once another workgroup has given
// up, it sets err and returns, so a grid that is not co-resident still ends.
__device__ __forceinline__ void barrier_wait(const PersistArgs& P, const uint32_t* c, uint32_t target) {
    uint32_t spins = 0;
    while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > P.spin_limit || __hip_atomic_load(P.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(P.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(32);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Grid barrier number `round` (1, 2, ...), in two levels over the XCDs the
// workgroups run on (s_xcd in LDS: the hardware XCD id, the workgroups on it
// and the XCDs with workgroups, counted at the launch's start).  Every
// workgroup waits until its own stores have reached its XCD's L2 (the vector
// L1 writes through) and counts in on its XCD's counter; the last to arrive
// writes that L2 back (a release at device scope, so the stores reach the
// other XCDs) and counts the XCD in: one write-back per XCD and barrier
// instead of one per workgroup, each of which would flush the whole L2 under
// the workgroups still computing.  All then wait for every XCD.
__device__ __forceinline__ void grid_barrier(const PersistArgs& P, uint32_t round, const uint32_t* s_xcd) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);                     // this wave's stores are in L2
    __syncthreads();
    if (threadIdx.x == 0) {
        // (read from LDS here rather than kept in registers across the tiles)
        const uint32_t xcc = s_xcd[0], members = s_xcd[1], groups = s_xcd[2];
        const uint32_t old = __hip_atomic_fetch_add(P.xbar + xcc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == round * members) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(P.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        barrier_wait(P, P.bar, groups * round);
    }
    __syncthreads();
}

// A run descriptor as workgroup-uniform values.  The kernel stores to memory,
// so the compiler cannot keep the descriptor loads scalar and would treat
// everything built from them (buffer resources, run constants) as per-lane
// values; every word is the same on all lanes, so the first lane's is taken.
__device__ __forceinline__ RunDesc uniform_desc(const RunDesc* p) {
    static_assert(sizeof(RunDesc) % 4 == 0, "descriptor words");
    RunDesc d;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
    uint32_t w[sizeof(RunDesc) / 4];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(RunDesc) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
    __builtin_memcpy(&d, w, sizeof(RunDesc));
    return d;
}

template <class St, class Tl>
__global__ __launch_bounds__(NTHR, (stage_min_waves<typename St::T, VAR_WENO>())) void persist_kernel(PersistArgs P) {
    const StageArgs& A = P.A;
    const int nall = A.tile_start[A.nruns];
    const int per = (nall + 7) / 8;
    const int G = (int)gridDim.x;
    // count the workgroups on each XCD (the hardware id; dispatch rotates the
    // XCD a block number lands on between launches), behind a one-level
    // barrier whose release writes back per workgroup
    __shared__ uint32_t s_xcd[3];
    if (threadIdx.x == 0) {
        const uint32_t xcc = __builtin_amdgcn_s_getreg(20 | (31 << 11)) & 7u;    // XCC_ID
        __hip_atomic_fetch_add(P.xreg + xcc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(P.xreg + 8, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        barrier_wait(P, P.xreg + 8, (uint32_t)G);
        uint32_t groups = 0;
        for (int i = 0; i < 8; ++i)
            groups += __hip_atomic_load(P.xreg + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        s_xcd[0] = xcc;
        s_xcd[1] = __hip_atomic_load(P.xreg + xcc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_xcd[2] = groups;
    }
    __syncthreads();
    uint32_t round = 0;
    for (int step = 0; step < P.nsteps; ++step) {
        for (int stage = 0; stage < 3; ++stage) {
            for (int vb = (int)blockIdx.x; vb < 8 * per; vb += G) {
                const int tg = (vb & 7) * per + (vb >> 3);
                if (tg < nall) {                       // uniform per workgroup
                    const int run = run_of(A, tg);
                    const RunDesc D = uniform_desc(A.desc[run] + stage);
                    const uint32_t ctr = sizeof(typename St::T) == 8 ? 0u : *D.ctr + (uint32_t)step;
                    // stage_tile even where per-stage launches take stage_tile_rounds
                    // (same bits): inside this loop the rounds kernel spills
                    stage_tile<St, Tl, VAR_WENO, 4, GN_RUNTIME>(A, D, tg - A.tile_start[run], ctr);
                }
                __syncthreads();                       // the tile's LDS is free again
            }
            grid_barrier(P, ++round, s_xcd);
        }
    }
    // after the last barrier every tile has read the step counters
    if (sizeof(typename St::T) != 8 && blockIdx.x == 0 && (int)threadIdx.x < A.nruns)
        const_cast<uint32_t*>(A.desc[threadIdx.x]->ctr)[0] += (uint32_t)P.nsteps;
}

__global__ __launch_bounds__(64) void persist_reset_kernel(uint32_t* bar) {
    if (threadIdx.x < PERSIST_WORDS) bar[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// Equilibrium initialisation: g_k = f^eq_k(rho, u, T) - w_k rho0 with the
// thermal order-2/3 Hermite terms for T != 1 (order 2 only for Q = 3),
// computed in FP64.
template <class St>
__global__ void init_kernel(const double* rho, const double* ut, const double* up,
                            const double* Tf, void* outv, Consts c, int n, double rho0) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    typename St::S* out = static_cast<typename St::S*>(outv);
    const double r = rho[i], a = ut[i], b = up[i];
    const double dT = Tf ? Tf[i] - 1.0 : 0.0;
    const double u2 = a * a + b * b;
    const int q = c.q;
    for (int k = 0; k < q * q; ++k) {
        const double vt = c.v[k / q], vp = c.v[k % q];
        const double xi = vt * a + vp * b, v2 = vt * vt + vp * vp;
        double pm1 = xi + 0.5 * (xi * xi - u2 + dT * (v2 - 2.0));
        if (q == 4) pm1 += xi * (xi * xi - 3.0 * u2 + 3.0 * dT * (v2 - 4.0)) / 6.0;
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
                                             int& nbad);

// Moment correction: f_k += f^eq_k(rho + d_rho, u + d_u) - f^eq_k(rho, u) with
// the isothermal equilibrium (eqs. (feq_Q=3), (feq_Q=4)); the non-equilibrium
// part of f is kept.
template <class St>
__global__ void correct_kernel(void* io, const double* drho, const double* dut, const double* dup,
                               Consts c, int n, double rho0) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    typename St::S* f = static_cast<typename St::S*>(io);
    double r, a, b, t, e;
    int nb;
    cell_moments<St>(f, i, n, c, rho0, r, a, b, t, e, nb);
    const double r2 = r + drho[i], a2 = a + dut[i], b2 = b + dup[i];
    const double u2 = a * a + b * b, w2 = a2 * a2 + b2 * b2;
    const int q = c.q;
    for (int k = 0; k < q * q; ++k) {
        const double vt = c.v[k / q], vp = c.v[k % q];
        const double x1 = vt * a + vp * b, x2 = vt * a2 + vp * b2;
        double p1 = x1 + 0.5 * (x1 * x1 - u2), p2 = x2 + 0.5 * (x2 * x2 - w2);
        if (q == 4) {
            p1 += x1 * (x1 * x1 - 3.0 * u2) / 6.0;
            p2 += x2 * (x2 * x2 - 3.0 * w2) / 6.0;
        }
        const size_t o = (size_t)k * n + i;
        const double g = (double)St::ld(f, o, c.iscale[k]) + c.wk[k] * ((r2 - r) + r2 * p2 - r * p1);
        St::st(f, o, (typename St::T)g, c.scale[k]);
    }
}

template <class St>
__device__ __forceinline__ void cell_moments(const typename St::S* in, size_t i, size_t n,
                                             const Consts& c, double rho0, double& rho,
                                             double& ut, double& up, double& T, double& e,
                                             int& nbad) {
    double g[NKMAX];
    double dr = 0, jt = 0, jp = 0;
    nbad = 0;
    const int q = c.q;
    for (int k = 0; k < q * q; ++k) {
        g[k] = (double)St::ld(in, (size_t)k * n + i, c.iscale[k]);
        nbad += isfinite(g[k]) ? 0 : 1;
        dr += g[k];
        jt += c.v[k / q] * g[k];
        jp += c.v[k % q] * g[k];
    }
    rho = rho0 + dr;
    ut = jt / rho;
    up = jp / rho;
    double th = 0, en = 0;
    for (int k = 0; k < q * q; ++k) {
        const double f = c.wk[k] * rho0 + g[k];
        const double vt = c.v[k / q], vp = c.v[k % q];
        const double dt_ = vt - ut, dp_ = vp - up;
        th += f * (dt_ * dt_ + dp_ * dp_);
        en += 0.5 * f * (vt * vt + vp * vp);
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

// One wavefront folds the per-block partials: lane l takes blocks l, l + 64,
// ... in order, then the 64 lane results are combined by a fixed pairwise
// tree in LDS, so the result depends only on the grid (deterministic).
__global__ __launch_bounds__(64) void reduce_final(const double* part, int nblk, double* out) {
    __shared__ double sh[8][64];
    const int l = threadIdx.x;
    double acc[8] = {0, 0, 0, 0, 0, 0, INFINITY, -INFINITY};
    for (int b = l; b < nblk; b += 64) {
        for (int j = 0; j < 5; ++j) acc[j] += part[(size_t)b * 8 + j];
        acc[5] = fmax(acc[5], part[(size_t)b * 8 + 5]);
        acc[6] = fmin(acc[6], part[(size_t)b * 8 + 6]);
        acc[7] = fmax(acc[7], part[(size_t)b * 8 + 7]);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) sh[j][l] = acc[j];
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (l < w) {
#pragma unroll
            for (int j = 0; j < 5; ++j) sh[j][l] += sh[j][l + w];
            sh[5][l] = fmax(sh[5][l], sh[5][l + w]);
            sh[6][l] = fmin(sh[6][l], sh[6][l + w]);
            sh[7][l] = fmax(sh[7][l], sh[7][l + w]);
        }
        __syncthreads();
    }
    if (l < 8) out[l] = sh[l][0];
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

// ---------------------------------------------------------------------------
// FP32 quadrature for the float kernels.  Rounded to FP32, the nodes and
// weights of the D2Q16 rule miss the moment identities of App. A (sum w = 1,
// sum w v^2 = 1, sum w v^4 = 3, sum w v_t^2 v_p^2 = 1) by 1e-8 .. 1e-7.  The
// BGK term then relaxes the mass and momentum toward slightly wrong values: a
// small force that acts every step and adds up over t / tau relaxation times.
// Two measures remove it:
//  - the FP32 nodes v_o = sqrt(3 + sqrt6), v_i = sqrt(3 - sqrt6) and the class
//    weights w_oo, w_oi, w_ii of the product rule are moved by a few ulps (nodes
//    10, weights 40; w_ii: the nearest floats to the mass identity): among the
//    candidates with sum w = 1 exactly, the one with the smallest
//    max(|S4 - 3|, 3 |S22 - 1|, |S4 - 3 S22|), S4 = sum w v_t^4, S22 = sum w
//    v_t^2 v_p^2 (about 2e-8 each, 2e-7 for the nearest floats);
//  - the equilibrium takes its coefficients from the rule's own moments (S2 =
//    sum w v_t^2): P(xi) = (1/S2) xi + (xi^2 - S2 u^2)/2 + xi (xi^2 - g u^2)/6
//    with g = (S4 + 3 S22) / (2 S2), which makes the mass and momentum of the
//    equilibrium exact for every u up to the remaining anisotropy S4 - 3 S22
//    (cubic in u).  For the FP64 rule these coefficients are 1, 1 and 3 up to
//    rounding.
// The mass and second-moment sums are evaluated exactly: every product of
// three floats is an integer multiple of 2^-100 below 2^127; the fourth moments
// in long double.
namespace quad32 {
constexpr int FXS = 100;
using i128 = __int128;
i128 exact(float a, float b = 1.f, float c = 1.f) {
    const float f[3] = {a, b, c};
    i128 m = 1;
    int q = 0;
    for (float x : f) {
        int e;
        const float fr = std::frexp(x, &e);
        m *= (i128)(int64_t)std::ldexp(fr, 24);
        q += e - 24;
    }
    const int sh = q + FXS;               // >= 0 for the magnitudes used here
    return m * ((i128)1 << sh);
}
float step_ulps(float x, int n) {
    for (int i = 0; i < (n < 0 ? -n : n); ++i) x = std::nextafter(x, n > 0 ? INFINITY : -INFINITY);
    return x;
}
double to_d(i128 x) { return std::ldexp((double)x, -FXS); }
struct Rule {
    float vo, vi, woo, woi, wii;
    double e00, e20;
    long double s2, s4, s22;
};
// n_out, n_in: outer and inner nodes per axis (Q = 4: 2 and 2; Q = 3: the
// nodes +-sqrt3 and the node 0, which stays exactly 0).  A population with m
// inner components has class weight w_{oo}, w_{oi}, w_{ii} for m = 0, 1, 2.
Rule search(int q) {
    const double r6 = std::sqrt(6.0);
    const double vo = q == 4 ? std::sqrt(3.0 + r6) : std::sqrt(3.0);
    const double vi = q == 4 ? std::sqrt(3.0 - r6) : 0.0;
    const int n_out = 2, n_in = q - 2;
    auto w1 = [&](double v) {
        const double h = q == 4 ? v * v * v * v * v - 10 * v * v * v + 15 * v : v * v * v * v - 6 * v * v + 3;
        return (q == 4 ? 24.0 : 6.0) / (h * h);
    };
    const double wo = w1(vo), wi = w1(vi);
    const i128 one = (i128)1 << FXS;
    constexpr int KU = 10, KW = 40;
    const int KI = q == 4 ? KU : 0;        // the zero node is exact
    Rule best{};
    double bestsc = -1;
    for (int a = -KU; a <= KU; ++a) {
        const float fvo = step_ulps((float)vo, a);
        const long double vo2 = (long double)fvo * fvo, vo4 = vo2 * vo2;
        for (int b = -KI; b <= KI; ++b) {
            const float fvi = step_ulps((float)vi, b);
            const long double vi2 = (long double)fvi * fvi, vi4 = vi2 * vi2;
            for (int c = -KW; c <= KW; ++c) {
                const float woo = step_ulps((float)(wo * wo), c);
                for (int d = -KW; d <= KW; ++d) {
                    const float woi = step_ulps((float)(wo * wi), d);
                    const float c0 = (float)((1.0 - n_out * n_out * (double)woo -
                                              2.0 * n_out * n_in * (double)woi) / (n_in * n_in));
                    for (int e = -1; e <= 1; ++e) {
                        const float wii = step_ulps(c0, e);
                        const i128 e00 = n_out * n_out * exact(woo) + 2 * n_out * n_in * exact(woi) +
                                         n_in * n_in * exact(wii) - one;
                        if (e00 != 0) continue;
                        const long double s4 = n_out * vo4 * (n_out * (long double)woo + n_in * (long double)woi) +
                                               n_in * vi4 * (n_out * (long double)woi + n_in * (long double)wii);
                        const long double s22 = n_out * n_out * (long double)woo * vo4 +
                                                2 * n_out * n_in * (long double)woi * vo2 * vi2 +
                                                n_in * n_in * (long double)wii * vi4;
                        const double e40 = (double)(s4 - 3), e22 = (double)(s22 - 1);
                        const double sc = std::fmax(std::fmax(std::fabs(e40), 3 * std::fabs(e22)),
                                                    std::fabs(e40 - 3 * e22));
                        if (bestsc < 0 || sc < bestsc) {
                            const i128 s20 = n_out * (n_out * exact(woo, fvo, fvo) + n_in * exact(woi, fvo, fvo)) +
                                             n_in * (n_out * exact(woi, fvi, fvi) + n_in * exact(wii, fvi, fvi));
                            bestsc = sc;
                            best = Rule{fvo, fvi, woo, woi, wii, to_d(e00), to_d(s20 - one)};
                            best.s2 = 1.0L + (long double)to_d(s20 - one);
                            best.s4 = s4;
                            best.s22 = s22;
                        }
                    }
                }
            }
        }
    }
    return best;
}
const Rule& rule(int q) {
    static const Rule r4 = search(4);
    static const Rule r3 = search(3);
    return q == 3 ? r3 : r4;
}
// FP32 nodes and weights of the rule for a population k = q kt + kp
inline void fp32_rule(int q, float v[NQMAX], float w[NKMAX]) {
    const Rule& r = rule(q);
    if (q == 4) {
        v[0] = -r.vo; v[1] = -r.vi; v[2] = r.vi; v[3] = r.vo;
    } else {
        v[0] = -r.vo; v[1] = 0.0f; v[2] = r.vo;
    }
    auto inner = [&](int i) { return (int)(q == 4 ? (i == 1 || i == 2) : i == 1); };
    const float cls[3] = {r.woo, r.woi, r.wii};
    for (int k = 0; k < q * q; ++k) w[k] = cls[inner(k / q) + inner(k % q)];
}
}  // namespace quad32

// Nodes (roots of H_Q: Q = 4, x^2 = 3 -+ sqrt6, App. A.2; Q = 3, x = 0, +-sqrt3,
// App. A.1), weights Q! / H_{Q+1}(v)^2, the kernels K^H, K~^H of eqs. (KH),
// (KtildeH) and the rank-1 force coefficients, all packed with stride Q.
void build_consts(Consts& c, int storage, int q) {
    c = Consts{};
    c.q = q;
    if (q == 4) {
        const double r6 = std::sqrt(6.0);
        c.v[0] = -std::sqrt(3.0 + r6);
        c.v[1] = -std::sqrt(3.0 - r6);
        c.v[2] = std::sqrt(3.0 - r6);
        c.v[3] = std::sqrt(3.0 + r6);
    } else {
        c.v[0] = -std::sqrt(3.0);
        c.v[1] = 0.0;
        c.v[2] = std::sqrt(3.0);
    }
    const double fact[NQMAX + 1] = {1.0, 1.0, 2.0, 6.0, 24.0};
    double w1[NQMAX];
    for (int i = 0; i < q; ++i) {
        const double h = hermite(q + 1, c.v[i]);
        w1[i] = fact[q] / (h * h);
    }
    for (int k = 0; k < q * q; ++k) c.wk[k] = w1[k / q] * w1[k % q];
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            double a = 0.0, b = 0.0;
            for (int l = 0; l < q; ++l) {
                const double hl1 = hermite(l + 1, c.v[i]) / fact[l];
                a += hl1 * hermite(l, c.v[j]);
                b += hl1 * (hermite(l + 1, c.v[j]) + l * hermite(l - 1, c.v[j]));
            }
            c.K[i * q + j] = -w1[i] * a;
            c.Kt[i * q + j] = -w1[i] * b;
        }
    // the rows of the nodes past the middle follow from the symmetric nodes
    // (H_n(-x) = (-1)^n H_n(x)): K^H[q-1-i][q-1-j] = -K^H[i][j] and
    // K~^H[q-1-i][q-1-j] = K~^H[i][j].  The recurrence already gives these
    // values; setting them makes the symmetry the stage kernel relies on exact.
    for (int i = (q + 1) / 2; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            c.K[i * q + j] = -c.K[(q - 1 - i) * q + (q - 1 - j)];
            c.Kt[i * q + j] = c.Kt[(q - 1 - i) * q + (q - 1 - j)];
        }
    for (int k = 0; k < q * q; ++k) {
        double sc = 1.0;
        if (storage == VLBM_STORE_F16_DEV) sc = std::ldexp(1.0, 10 - (int)std::lround(std::log2(c.wk[k])));
        c.scale[k] = sc;
        c.iscale[k] = 1.0 / sc;
    }
}

// Rest-state tables for a grid.  With g = 0 the populations are w_k rho0.  The
// theta flux of the rest state at an interface is v_k w_k rho0 times the WENO
// combination of the candidates C1, C2, C3 of S_j = sin(theta_j):
//   C2 + w1 (C1 - C2) + w3 (C3 - C2),
// where the weights are those of the actual data (the indicators of g).  The
// C2 part and the inertial force on w_k rho0 are exact per row and go into
// rest[] (times dt); the kernel adds w1 (C1 - C2) + w3 (C3 - C2) from dC.
struct HostRows {
    std::vector<double> sinv, sgeo, inv_sdth, inv_sdph, cot, rest, dC, sI;
};

void build_rows(HostRows& h, const vlbm_params& p, const Consts& c) {
    const int nt = p.n_theta, np = p.n_phi;
    const double dth = M_PI / nt, dph = 2.0 * M_PI / np, R = p.radius;
    const int scheme = p.advection & VLBM_ADV_SCHEME_MASK;
    const bool kom = (p.advection & VLBM_ADV_KOMISSAROV) != 0;
    // theta flux function V f = v S_j f: S_j = sin th_j (signed in ghost rows), or
    // 1 in the Komissarov form, eq. (Komissarov_scheme), whose interface flux is
    // then multiplied by sin th_{i-1/2} (the angle to the nearer pole, so both
    // pole values are 0) and divided by R (cos th_{s-1/2} - cos th_{s+1/2})
    h.sinv.resize(nt + 2 * NGH);
    for (int j = -NGH; j < nt + NGH; ++j) h.sinv[j + NGH] = kom ? 1.0 : std::sin((j + 0.5) * dth);
    // the geometry itself (area element, vorticity), whatever the flux form
    h.sgeo.resize(nt + 2 * NGH);
    for (int j = -NGH; j < nt + NGH; ++j) h.sgeo[j + NGH] = std::sin((j + 0.5) * dth);
    h.sI.resize(nt + 1);
    for (int i = 0; i <= nt; ++i) h.sI[i] = kom ? std::sin((i < nt - i ? i : nt - i) * dth) : 1.0;
    h.inv_sdth.resize(nt);
    h.inv_sdph.resize(nt);
    h.cot.resize(nt);
    for (int s = 0; s < nt; ++s) {
        const double th = (s + 0.5) * dth;
        h.inv_sdth[s] = kom ? 1.0 / (R * (std::cos(s * dth) - std::cos((s + 1) * dth)))
                            : 1.0 / (R * std::sin(th) * dth);
        h.inv_sdph[s] = 1.0 / (R * std::sin(th) * dph);
        h.cot[s] = std::cos(th) / (R * std::sin(th));
    }
    // reconstructions of S_j at interface i (= s + 1/2, s = i - 1): the rest
    // state's flux (WENO: central candidate C2, whose weights the kernel adds
    // through C1 - C2 and C3 - C2; upwind schemes: their fixed stencil)
    h.dC.assign(2 * (nt + 1) * 2, 0.0);
    std::vector<double> c2(2 * (nt + 1));
    for (int dir = 0; dir < 2; ++dir)
        for (int i = 0; i <= nt; ++i) {
            const int s = i - 1;
            double P[5];
            for (int m = 0; m < 5; ++m) {
                const int j = dir == 0 ? s - 2 + m : s + 3 - m;   // mirrored stencil
                P[m] = h.sinv[j + NGH];
            }
            double rec;
            if (kom) {
                rec = 1.0;              // every scheme reconstructs a constant exactly
            } else if (scheme == VLBM_ADV_WENO5) {
                const double C1 = P[0] / 3.0 - 7.0 * P[1] / 6.0 + 11.0 * P[2] / 6.0;
                const double C2 = -P[1] / 6.0 + 5.0 * P[2] / 6.0 + P[3] / 3.0;
                const double C3 = P[2] / 3.0 + 5.0 * P[3] / 6.0 - P[4] / 6.0;
                h.dC[(dir * (nt + 1) + i) * 2 + 0] = p.rho0 * (C1 - C2);
                h.dC[(dir * (nt + 1) + i) * 2 + 1] = p.rho0 * (C3 - C2);
                rec = C2;
            } else if (scheme == VLBM_ADV_U1) {
                rec = P[2];
            } else if (scheme == VLBM_ADV_U2) {
                rec = 1.5 * P[2] - 0.5 * P[1];
            } else {
                rec = P[3] / 3.0 + 5.0 * P[2] / 6.0 - P[1] / 6.0;
            }
            c2[dir * (nt + 1) + i] = rec * h.sI[i];
        }
    const int q = c.q;
    h.rest.assign((size_t)q * q * nt, 0.0);
    const double r0 = p.rho0;
    for (int k = 0; k < q * q; ++k) {
        const int kt = k / q, kp = k % q;
        const int dir = c.v[kt] > 0 ? 0 : 1;
        for (int s = 0; s < nt; ++s) {
            const double vw = c.v[kt] * c.wk[k] * r0;
            const double adv = -h.inv_sdth[s] * vw * (c2[dir * (nt + 1) + s + 1] - c2[dir * (nt + 1) + s]);
            double dfdvt = 0.0, dfvdvp = 0.0;
            for (int b = 0; b < q; ++b) {
                dfdvt += c.K[kt * q + b] * c.wk[b * q + kp] * r0;
                dfvdvp += c.Kt[kp * q + b] * c.wk[kt * q + b] * r0;
            }
            const double G = -h.cot[s] * (c.v[kp] * c.v[kp] * dfdvt - c.v[kt] * dfvdvp);
            h.rest[(size_t)k * nt + s] = p.dt * (adv + G);
        }
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

size_t store_bytes(int storage) {
    return storage == VLBM_STORE_F64 ? 8 : storage == VLBM_STORE_F32_DEV ? 4 : 2;
}

constexpr int RED_BLOCKS = 1024;

struct Layout {
    size_t fbuf[3], sinv, sinv_f, sgeo, inv_sdth, inv_sdph, cot, rest, rest_f, dC, sI, rowk, rowk_f, facek, facek_f;
    size_t fields, part, dout, desc, ctr, bar, total;
};

Layout layout_of(const vlbm_params& p) {
    Layout L{};
    const size_t n = (size_t)p.n_theta * p.n_phi;
    size_t off = 0;
    const size_t nk = (size_t)p.q * p.q;
    const size_t fb = align_up(nk * n * store_bytes(p.storage));
    for (int i = 0; i < 3; ++i) { L.fbuf[i] = off; off += fb; }
    L.sinv = off; off += align_up(sizeof(double) * (p.n_theta + 2 * NGH));
    L.sgeo = off; off += align_up(sizeof(double) * (p.n_theta + 2 * NGH));
    L.sinv_f = off; off += align_up(sizeof(float) * (p.n_theta + 2 * NGH));
    L.inv_sdth = off; off += align_up(sizeof(double) * p.n_theta);
    L.inv_sdph = off; off += align_up(sizeof(double) * p.n_theta);
    L.cot = off; off += align_up(sizeof(double) * p.n_theta);
    L.rest = off; off += align_up(sizeof(double) * nk * p.n_theta);
    L.rest_f = off; off += 3 * align_up(sizeof(float) * nk * p.n_theta);    // per stage
    L.dC = off; off += align_up(sizeof(double) * 4 * (p.n_theta + 1));
    L.sI = off; off += align_up(sizeof(double) * (p.n_theta + 1));
    L.rowk = off; off += align_up(sizeof(CellRowK<double>) * p.n_theta);
    L.rowk_f = off; off += 3 * align_up(sizeof(CellRowK<float>) * p.n_theta);   // per stage
    L.facek = off; off += align_up(sizeof(FaceRowK<double>) * (p.n_theta + 1));
    L.facek_f = off; off += align_up(sizeof(FaceRowK<float>) * (p.n_theta + 1));
    L.fields = off; off += align_up(sizeof(double) * 4 * n);
    L.part = off; off += align_up(sizeof(double) * 8 * RED_BLOCKS);
    L.dout = off; off += align_up(sizeof(double) * 8);
    L.desc = off; off += align_up(sizeof(RunDesc) * 3);
    L.ctr = off; off += align_up(sizeof(uint32_t));
    L.bar = off; off += align_up(PERSIST_WORDS * sizeof(uint32_t));   // persistent launch: barrier state
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
    if (p->q != 3 && p->q != 4)
        return fail(VLBM_ERR_UNSUPPORTED, "q = %d: the quadratures are q = 3 (D2Q9) and 4 (D2Q16)", p->q);
    if (p->storage >= 0 && p->storage <= 2 &&
        (unsigned long long)p->q * p->q * p->n_theta * p->n_phi * store_bytes(p->storage) > 0xffffffffULL)
        return fail(VLBM_ERR_UNSUPPORTED,
                    "one population buffer must stay below 4 GiB (32-bit buffer offsets)");
    if (!(p->radius > 0) || !(p->tau > 0) || !(p->dt > 0) || !(p->rho0 > 0) || !(p->weno_eps > 0))
        return fail(VLBM_ERR_ARG, "radius, tau, dt, rho0 and weno_eps must be > 0");
    if (!std::isfinite(p->radius) || !std::isfinite(p->tau) || !std::isfinite(p->dt) ||
        !std::isfinite(p->rho0) || !std::isfinite(p->weno_eps))
        return fail(VLBM_ERR_ARG, "non-finite parameter");

    if (p->storage < 0 || p->storage > 2) return fail(VLBM_ERR_UNSUPPORTED, "unknown storage %d", p->storage);
    if ((p->advection & ~(VLBM_ADV_SCHEME_MASK | VLBM_ADV_KOMISSAROV)) ||
        (p->advection & VLBM_ADV_SCHEME_MASK) > VLBM_ADV_U3)
        return fail(VLBM_ERR_UNSUPPORTED, "unknown advection %d", p->advection);
    return VLBM_OK;
}

}  // namespace

struct vlbm_ctx {
    vlbm_params p;
    hipStream_t stream;
    char* ws;
    Layout L;
    Consts c;
    ConstsT<double> cd;
    ConstsT<float> cf;
    int64_t launches;
    int device;
    int tile;       // 0: 15 x 16 tiles, 1: 7 x 32
};

struct vlbm_graph {
    std::vector<vlbm_ctx*> ctxs;
    std::vector<const uint32_t*> errs;   // persistent graphs: the barrier error flag of each launch group
    int64_t steps = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~vlbm_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
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

template <class F>
vlbm_status dispatch(int storage, F&& f) {
    switch (storage) {
        case VLBM_STORE_F64: return f(StF64{});
        case VLBM_STORE_F32_DEV: return f(StF32{});
        default: return f(StF16{});
    }
}

const RunDesc* desc_of(vlbm_ctx* x, int stage) {
    return reinterpret_cast<const RunDesc*>(x->ws + x->L.desc) + (stage - 1);
}

// The three per-stage descriptors of a context (stage 3 writes over f_n).
void fill_descs(vlbm_ctx* x, RunDesc d[3]) {
    void* fn = x->ws + x->L.fbuf[0];
    void* fa = x->ws + x->L.fbuf[1];
    void* fb = x->ws + x->L.fbuf[2];
    for (int i = 0; i < 3; ++i) {
        RunDesc& D = d[i];
        D.rows.sinv = at<double>(x, x->L.sinv);
        D.rows.inv_sdth = at<double>(x, x->L.inv_sdth);
        D.rows.inv_sdph = at<double>(x, x->L.inv_sdph);
        D.rows.cot = at<double>(x, x->L.cot);
        D.rows.rest = at<double>(x, x->L.rest);
        D.rows.dC = at<double>(x, x->L.dC);
        D.rows.sI = at<double>(x, x->L.sI);
        D.scheme = x->p.advection & VLBM_ADV_SCHEME_MASK;
        D.rest_f = at<float>(x, x->L.rest_f + i * align_up(sizeof(float) * x->p.q * x->p.q * x->p.n_theta));
        D.sinv_f = at<float>(x, x->L.sinv_f);
        D.nt = x->p.n_theta;
        D.np = x->p.n_phi;
        D.dt = x->p.dt;
        D.inv_tau = 1.0 / x->p.tau;
        D.rho0 = x->p.rho0;
        D.eps = x->p.weno_eps;
        D.gn = fn;
        D.ctr = at<uint32_t>(x, x->L.ctr);
        D.seq = 16u * (uint32_t)i;
        const bool f64 = x->p.storage == VLBM_STORE_F64;
        D.rowk = f64 ? static_cast<const void*>(at<CellRowK<double>>(x, x->L.rowk))
                     : static_cast<const void*>(at<CellRowK<float>>(
                           x, x->L.rowk_f + i * align_up(sizeof(CellRowK<float>) * x->p.n_theta)));
        D.facek = f64 ? static_cast<const void*>(at<FaceRowK<double>>(x, x->L.facek))
                      : static_cast<const void*>(at<FaceRowK<float>>(x, x->L.facek_f));
    }
    d[0].gin = fn; d[0].out = fa;
    d[1].gin = fa; d[1].out = fb;
    d[2].gin = fb; d[2].out = fn;
    for (int i = 0; i < 3; ++i) { d[i].a = RK_A[i]; d[i].b = RK_B[i]; }
    for (int i = 0; i < 3; ++i) {
        RunDesc& D = d[i];
        D.ud[U_DTI] = D.dt * D.inv_tau;
        D.ud[U_EPSK] = 12.0 / 13.0 * D.eps;
        D.ud[U_OMDTI] = 1.0 - D.ud[U_DTI];
        D.ud[U_RHO0] = D.rho0;
        D.ud[U_A] = D.a;
        D.ud[U_B] = D.b;
        for (int j = 0; j < U_N; ++j) D.uf[j] = (float)D.ud[j];
        D.uf[U_DTI] = (float)(D.b * D.ud[U_DTI]);
    }
}

// The kernel variant a context's scheme needs.
template <class St>
int variant_of(const vlbm_ctx* x) {
    const int scheme = x->p.advection & VLBM_ADV_SCHEME_MASK;
    if (scheme != VLBM_ADV_WENO5) return VAR_UPWIND;
    return (x->p.advection != VLBM_ADV_WENO5 || x->p.q == 3) ? VAR_WENO_GEN : VAR_WENO;
}

// One launch of one variant over up to MAXRUNS contexts.
template <class St, int VAR>
vlbm_status launch_group(vlbm_ctx* const* xs, int m, int stage, hipStream_t stream) {
    StageArgs A;
    A.cd = xs[0]->cd;
    A.cf = xs[0]->cf;
    A.nruns = m;
    A.tile_start[0] = 0;
    for (int i = 0; i < m; ++i) {
        vlbm_ctx* x = xs[i];
        A.desc[i] = desc_of(x, stage);
        A.tile_start[i + 1] = A.tile_start[i] + n_tiles(x->p.n_theta, x->p.n_phi, x->tile);
        x->launches++;
    }
    const int nb = A.tile_start[m];
    const dim3 grid(8 * ((nb + 7) / 8));
    const bool wide = xs[0]->tile == 1;
    const bool d2q9 = xs[0]->p.q == 3;
    if (m == 1) {
        RunDesc d[3];
        fill_descs(xs[0], d);
        A.run0 = d[stage - 1];
    }
    // stage 1 runs the copy without the step input g_n, stages 2 and 3 the
    // copy that combines with it
    auto go = [&](auto batch, auto tl) {
        constexpr bool BT = decltype(batch)::value;
        using TL = decltype(tl);
        auto launch = [&](auto gn) {
            constexpr int GN = decltype(gn)::value;
            if constexpr (VAR == VAR_WENO) {
                hipLaunchKernelGGL((stage_kernel<St, BT, TL, VAR_WENO, 4, false, GN>), grid, dim3(NTHR), 0, stream, A);
            } else {
                if (d2q9) hipLaunchKernelGGL((stage_kernel<St, BT, TL, VAR, 3, false, GN>), grid, dim3(NTHR), 0, stream, A);
                else hipLaunchKernelGGL((stage_kernel<St, BT, TL, VAR, 4, false, GN>), grid, dim3(NTHR), 0, stream, A);
            }
        };
        if (stage == 1) launch(std::integral_constant<int, GN_NONE>{});
        else launch(std::integral_constant<int, GN_LOAD>{});
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    // a single FP32 run of at least 2048 15 x 16 tiles takes the rounds
    // kernel's direct-to-LDS form, which pays off on large grids only
    // (single-run MLUPS against the register form: 256 x 512 -3.6 %,
    // 512 x 1024 and 1024 x 2048 equal, 1536 x 3072 +1.1 %, 2048 x 4096 +0.5 %)
    constexpr int DMA_MIN_TILES = 2048;
    if constexpr (std::is_same<St, StF32>::value && (VAR == VAR_WENO || VAR == VAR_UPWIND)) {
        if (m == 1 && !wide && !d2q9 && nb >= DMA_MIN_TILES) {
            if (stage == 1)
                hipLaunchKernelGGL((stage_kernel<St, false, Tile15x16, VAR, 4, true, GN_NONE>), grid, dim3(NTHR), 0, stream, A);
            else
                hipLaunchKernelGGL((stage_kernel<St, false, Tile15x16, VAR, 4, true, GN_LOAD>), grid, dim3(NTHR), 0, stream, A);
            return launch_check();
        }
    }
    if (m == 1) { if (wide) go(F_{}, Tile7x32{}); else go(F_{}, Tile15x16{}); }
    else { if (wide) go(T_{}, Tile7x32{}); else go(T_{}, Tile15x16{}); }
    return launch_check();
}

// One RK stage for n contexts of the same storage format: one launch per
// kernel variant present, MAXRUNS contexts per launch.
template <class St>
vlbm_status launch_stage(vlbm_ctx* const* xs, int n, int stage, hipStream_t stream) {
    static_assert(sizeof(StageArgs) <= 4096, "kernel arguments must fit the 4 KiB kernarg segment");
    std::vector<vlbm_ctx*> by[3];
    for (int i = 0; i < n; ++i) by[variant_of<St>(xs[i])].push_back(xs[i]);
    for (int v = 0; v < 3; ++v)
        for (size_t c0 = 0; c0 < by[v].size(); c0 += MAXRUNS) {
            const int m = (int)std::min<size_t>(MAXRUNS, by[v].size() - c0);
            vlbm_ctx* const* g = by[v].data() + c0;
            vlbm_status st = v == VAR_WENO ? launch_group<St, VAR_WENO>(g, m, stage, stream)
                           : v == VAR_WENO_GEN ? launch_group<St, VAR_WENO_GEN>(g, m, stage, stream)
                                               : launch_group<St, VAR_UPWIND>(g, m, stage, stream);
            if (st) return st;
        }
    return VLBM_OK;
}

// Advance the step counters (dither phase of the reduced-precision stores) of
// the contexts of one launch group, after their third stage.
struct CtrArgs {
    uint32_t* p[MAXRUNS];
    int n;
};
__global__ __launch_bounds__(64) void count_step_kernel(CtrArgs a) {
    const int i = threadIdx.x;
    if (i < a.n) a.p[i][0] += 1u;
}

vlbm_status count_steps(vlbm_ctx* const* xs, int n, hipStream_t stream) {
    for (int c0 = 0; c0 < n; c0 += MAXRUNS) {
        CtrArgs a{};
        a.n = n - c0 < MAXRUNS ? n - c0 : MAXRUNS;
        for (int i = 0; i < a.n; ++i) a.p[i] = at<uint32_t>(xs[c0 + i], xs[c0 + i]->L.ctr);
        hipLaunchKernelGGL(count_step_kernel, dim3(1), dim3(64), 0, stream, a);
        vlbm_status st = launch_check();
        if (st) return st;
    }
    return VLBM_OK;
}

vlbm_status check_batch(vlbm_ctx* const* xs, int n) {
    if (!xs || n < 1) return fail(VLBM_ERR_ARG, "empty context list");
    for (int i = 0; i < n; ++i) {
        if (!xs[i]) return fail(VLBM_ERR_ARG, "NULL context %d", i);
        if (xs[i]->p.storage != xs[0]->p.storage)
            return fail(VLBM_ERR_ARG, "contexts of a batch must share the storage format");
        if (xs[i]->stream != xs[0]->stream)
            return fail(VLBM_ERR_ARG, "contexts of a batch must share the stream");
        if (xs[i]->device != xs[0]->device)
            return fail(VLBM_ERR_ARG, "contexts of a batch must share the device");
        if (xs[i]->tile != xs[0]->tile)
            return fail(VLBM_ERR_ARG, "contexts of a batch must share the tile shape");
        if (xs[i]->p.q != xs[0]->p.q)
            return fail(VLBM_ERR_ARG, "contexts of a batch must share the quadrature order");
        for (int j = 0; j < i; ++j)
            if (xs[j] == xs[i]) return fail(VLBM_ERR_ARG, "context %d appears twice", i);
    }
    return VLBM_OK;
}

vlbm_status step_batch(vlbm_ctx* const* xs, int n, int64_t n_steps, hipStream_t stream) {
    for (int64_t i = 0; i < n_steps; ++i) {
        for (int stage = 1; stage <= 3; ++stage) {
            vlbm_status st = dispatch(xs[0]->p.storage, [&](auto tag) {
                return launch_stage<decltype(tag)>(xs, n, stage, stream);
            });
            if (st) return st;
        }
        if (xs[0]->p.storage != VLBM_STORE_F64) {
            vlbm_status st = count_steps(xs, n, stream);
            if (st) return st;
        }
    }
    return VLBM_OK;
}

// Polls of one grid-barrier wait before the persistent kernel gives up (about
// a second at the default; a stage takes about a millisecond).
uint32_t g_spin_limit = 1u << 20;

// Persistent stepping of up to MAXRUNS contexts of one storage format (WENO-5
// standard form, Q = 4).  Synchronous: waits for the launch to read the
// barrier's error flag.
// recording: the launches go into a HIP graph being captured on stream; they
// are then ordinary kernel nodes (co-resident by the grid size when nothing
// else runs on the device), and the error flag is read by vlbm_graph_check.
template <class St>
vlbm_status persist_group(vlbm_ctx* const* xs, int m, int64_t nsteps, hipStream_t stream, bool recording) {
    PersistArgs P{};
    StageArgs& A = P.A;
    A.cd = xs[0]->cd;
    A.cf = xs[0]->cf;
    A.nruns = m;
    A.tile_start[0] = 0;
    for (int i = 0; i < m; ++i) {
        A.desc[i] = desc_of(xs[i], 1);
        A.tile_start[i + 1] = A.tile_start[i] + n_tiles(xs[i]->p.n_theta, xs[i]->p.n_phi, xs[i]->tile);
    }
    const int nall = A.tile_start[m];
    const void* fn = xs[0]->tile == 1 ? reinterpret_cast<const void*>(persist_kernel<St, Tile7x32>)
                                      : reinterpret_cast<const void*>(persist_kernel<St, Tile15x16>);
    // co-resident workgroups: the runtime's occupancy, capped by the LDS a CU
    // was measured to hold for five 32 KiB workgroups (not all of its 160 KiB)
    int ncu = 0, occ = 0;
    HIP_OK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, xs[0]->device));
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, NTHR, 0));
    hipFuncAttributes fa{};
    HIP_OK(hipFuncGetAttributes(&fa, fn));
    if (fa.sharedSizeBytes > 0) occ = std::min<int>(occ, (int)(159744 / fa.sharedSizeBytes));
    const int per = (nall + 7) / 8;
    const int G = std::min(8 * ((occ * ncu) / 8), 8 * per);
    if (G < 8) return fail(VLBM_ERR_DEVICE, "no co-resident grid for the persistent stage kernel");
    P.bar = at<uint32_t>(xs[0], xs[0]->L.bar);
    P.err = P.bar + 1;
    P.xbar = P.bar + 2;
    P.xreg = P.bar + 10;
    P.spin_limit = g_spin_limit;
    // one launch carries at most as many steps as the 32-bit arrival counts allow
    const int64_t chunk = std::min<int64_t>(INT32_MAX, (int64_t)(0xffffffffu / (3u * (uint32_t)G)));
    for (int64_t done = 0; done < nsteps;) {
        P.nsteps = (int)std::min(nsteps - done, chunk);
        hipLaunchKernelGGL(persist_reset_kernel, dim3(1), dim3(64), 0, stream, P.bar);
        vlbm_status st = launch_check();
        if (st) return st;
        void* args[] = {&P};
        if (recording) {
            HIP_OK(hipLaunchKernel(fn, dim3(G), dim3(NTHR), args, 0, stream));
            done += P.nsteps;
            continue;
        }
        HIP_OK(hipLaunchCooperativeKernel(fn, dim3(G), dim3(NTHR), args, 0, stream));
        HIP_OK(hipStreamSynchronize(stream));
        uint32_t err = 0;
        HIP_OK(hipMemcpy(&err, P.err, sizeof(err), hipMemcpyDeviceToHost));
        if (err)
            return fail(VLBM_ERR_DEVICE, "persistent stepping: a grid barrier wait gave up after %u polls; "
                        "the runs' state is undefined", P.spin_limit);
        done += P.nsteps;
    }
    if (!recording)
        for (int i = 0; i < m; ++i) xs[i]->launches += 3 * nsteps;
    return VLBM_OK;
}

// Persistent stepping of contexts already checked by check_batch.
vlbm_status step_persistent(vlbm_ctx* const* xs, int n, int64_t n_steps, hipStream_t stream, bool recording) {
    for (int i = 0; i < n; ++i)
        if (xs[i]->p.q != 4 || xs[i]->p.advection != VLBM_ADV_WENO5)
            return fail(VLBM_ERR_ARG, "persistent stepping needs D2Q16 with the standard WENO-5 form (context %d)", i);
    if (n_steps == 0) return VLBM_OK;
    for (int c0 = 0; c0 < n; c0 += MAXRUNS) {
        const int m = std::min(MAXRUNS, n - c0);
        vlbm_status st = dispatch(xs[0]->p.storage, [&](auto tag) {
            return persist_group<decltype(tag)>(xs + c0, m, n_steps, stream, recording);
        });
        if (st) return st;
    }
    return VLBM_OK;
}

vlbm_status copy_in(vlbm_ctx* x, double* dst, const double* src, size_t n, int on_dev) {
    HIP_OK(hipMemcpyAsync(dst, src, n * sizeof(double),
                          on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, x->stream));
    return VLBM_OK;
}

}  // namespace

// error text shared with closure.hip (not exported)
__attribute__((visibility("hidden"))) vlbm_status vlbm_set_error(vlbm_status st, const char* msg) {
    return fail(st, "%s", msg);
}

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

vlbm_status vlbm_set_tile_shape(vlbm_ctx* x, int rows, int cols) {
    if (!x) return fail(VLBM_ERR_ARG, "NULL context");
    for (int i = 0; i < 2; ++i)
        if (rows == TILE_ROWS[i] && cols == TILE_COLS[i]) {
            x->tile = i;
            return VLBM_OK;
        }
    return fail(VLBM_ERR_UNSUPPORTED, "tile shape %dx%d (supported: 15x16, 7x32)", rows, cols);
}

vlbm_status vlbm_quadrature_f32(float v[4], float w[16], double residual[4]) {
    if (!v || !w || !residual) return fail(VLBM_ERR_ARG, "NULL output");
    quad32::fp32_rule(4, v, w);
    const quad32::Rule& r = quad32::rule(4);
    residual[0] = r.e00;
    residual[1] = r.e20;
    residual[2] = (double)(r.s4 - 3.0L);
    residual[3] = (double)(r.s22 - 1.0L);
    return VLBM_OK;
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
    x->tile = 0;
    build_consts(x->c, p->storage, p->q);
    const int q = p->q;
    float fv[NQMAX] = {}, fw[NKMAX] = {};
    quad32::fp32_rule(q, fv, fw);
    for (int i = 0; i < q; ++i) { x->cd.v[i] = x->c.v[i]; x->cf.v[i] = fv[i]; }
    {
        // moments of the FP64 rule and of the FP32 rule, evaluated exactly enough
        long double d2 = 0, d4 = 0, d22 = 0;
        for (int k = 0; k < q * q; ++k) {
            const long double a = x->c.v[k / q], b = x->c.v[k % q], wk = x->c.wk[k];
            d2 += wk * a * a; d4 += wk * a * a * a * a; d22 += wk * a * a * b * b;
        }
        const quad32::Rule& r = quad32::rule(q);
        x->cd.eq_e1 = (double)(1.0L / d2 - 1.0L);
        x->cd.eq_hb = (double)(-0.5L * d2);
        x->cd.eq_g6 = (double)((d4 + 3.0L * d22) / (12.0L * d2));
        x->cf.eq_e1 = (float)(1.0L / r.s2 - 1.0L);
        x->cf.eq_hb = (float)(-0.5L * r.s2);
        x->cf.eq_g6 = (float)((r.s4 + 3.0L * r.s22) / (12.0L * r.s2));
    }
    for (int k = 0; k < q * q; ++k) {
        const double vw = x->c.v[k / q] * x->c.wk[k];
        x->cd.wk[k] = x->c.wk[k]; x->cf.wk[k] = fw[k];
        x->cd.wr[k] = x->c.wk[k];
        x->cf.wr[k] = fv[k / q] != 0.f ? (float)(vw / (double)fv[k / q]) : 0.f;
        x->cd.scale[k] = x->c.scale[k]; x->cf.scale[k] = (float)x->c.scale[k];
        x->cd.iscale[k] = x->c.iscale[k]; x->cf.iscale[k] = (float)x->c.iscale[k];
    }
    for (int i = 0; i < q * q; ++i) {
        x->cd.K[i] = x->c.K[i]; x->cf.K[i] = (float)x->c.K[i];
        x->cd.Kt[i] = x->c.Kt[i]; x->cf.Kt[i] = (float)x->c.Kt[i];
    }
    for (int i = 0; i < q; ++i) {
        x->cd.nv2[i] = -x->c.v[i] * x->c.v[i];
        x->cf.nv2[i] = (float)(-x->c.v[i] * x->c.v[i]);
    }
    HostRows h;
    build_rows(h, *p, x->c);
    // float kernels: the rest table and row factors of stage i times its b
    std::vector<float> rest_f(3 * h.rest.size());
    for (int i = 0; i < 3; ++i)
        for (size_t j = 0; j < h.rest.size(); ++j) rest_f[i * h.rest.size() + j] = (float)(RK_B[i] * h.rest[j]);
    // the stage kernel's per-row constants in both arithmetic types
    const int nt = p->n_theta;
    const double fsc = (p->advection & VLBM_ADV_SCHEME_MASK) == VLBM_ADV_WENO5 ? 1.0 / 6.0 : 1.0;
    const double vod = x->c.v[q - 1], vid = q == 4 ? x->c.v[q / 2] : 0.0;
    const double vof = fv[q - 1], vif = q == 4 ? fv[q / 2] : 0.0;
    std::vector<CellRowK<double>> rkd(nt);
    std::vector<CellRowK<float>> rkf(3 * nt);
    for (int s = 0; s < nt; ++s) {
        const double dth = p->dt * h.inv_sdth[s] * fsc, dph = p->dt * h.inv_sdph[s] * fsc;
        const double dc = p->dt * h.cot[s];
        rkd[s] = {vod * dth, vid * dth, vod * dph, vid * dph, dc, {0.0, 0.0, 0.0}};
        for (int i = 0; i < 3; ++i) {
            const double b = RK_B[i];
            rkf[i * nt + s] = {(float)(b * vof * dth), (float)(b * vif * dth), (float)(b * vof * dph),
                               (float)(b * vif * dph), (float)(b * dc), {0.f, 0.f, 0.f}};
        }
    }
    std::vector<FaceRowK<double>> fkd(nt + 1);
    std::vector<FaceRowK<float>> fkf(nt + 1);
    for (int i = 0; i <= nt; ++i) {
        const double* pp = &h.dC[2 * i];
        const double* pm = &h.dC[2 * (nt + 1) + 2 * i];
        fkd[i] = {3.0 * pp[0], 6.0 * pp[1], 3.0 * pm[0], 6.0 * pm[1], h.sI[i], {0.0, 0.0, 0.0}};
        fkf[i] = {(float)(3.0 * pp[0]), (float)(6.0 * pp[1]), (float)(3.0 * pm[0]),
                  (float)(6.0 * pm[1]), (float)h.sI[i], {0.f, 0.f, 0.f}};
    }
    hipError_t e = hipGetDevice(&x->device);
    const struct { size_t off; const std::vector<double>* v; } up[] = {
        {L.sinv, &h.sinv}, {L.sgeo, &h.sgeo}, {L.inv_sdth, &h.inv_sdth}, {L.inv_sdph, &h.inv_sdph},
        {L.cot, &h.cot}, {L.rest, &h.rest}, {L.dC, &h.dC}, {L.sI, &h.sI}};
    for (const auto& u : up) {
        if (e != hipSuccess) break;
        e = hipMemcpyAsync(x->ws + u.off, u.v->data(), u.v->size() * sizeof(double),
                           hipMemcpyHostToDevice, x->stream);
    }
    // the per-stage float tables sit 256-byte aligned, one after the other
    std::vector<float> sinv_f(h.sinv.begin(), h.sinv.end());
    const size_t nrest = h.rest.size();
    const size_t rest_stride = align_up(sizeof(float) * nrest);
    const size_t rowk_stride = align_up(sizeof(CellRowK<float>) * nt);
    const struct { size_t off; const void* src; size_t bytes; } upk[] = {
        {L.rest_f, rest_f.data(), nrest * sizeof(float)},
        {L.rest_f + rest_stride, rest_f.data() + nrest, nrest * sizeof(float)},
        {L.rest_f + 2 * rest_stride, rest_f.data() + 2 * nrest, nrest * sizeof(float)},
        {L.rowk, rkd.data(), rkd.size() * sizeof(rkd[0])},
        {L.rowk_f, rkf.data(), nt * sizeof(rkf[0])},
        {L.rowk_f + rowk_stride, rkf.data() + nt, nt * sizeof(rkf[0])},
        {L.rowk_f + 2 * rowk_stride, rkf.data() + 2 * nt, nt * sizeof(rkf[0])},
        {L.facek, fkd.data(), fkd.size() * sizeof(fkd[0])},
        {L.facek_f, fkf.data(), fkf.size() * sizeof(fkf[0])},
        {L.sinv_f, sinv_f.data(), sinv_f.size() * sizeof(float)}};
    for (const auto& u : upk)
        if (e == hipSuccess)
            e = hipMemcpyAsync(x->ws + u.off, u.src, u.bytes, hipMemcpyHostToDevice, x->stream);
    RunDesc descs[3];
    fill_descs(x, descs);
    const uint32_t zero = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(x->ws + L.desc, descs, sizeof(descs), hipMemcpyHostToDevice, x->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(x->ws + L.ctr, &zero, sizeof(zero), hipMemcpyHostToDevice, x->stream);
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
    return step_batch(&x, 1, n_steps, x->stream);
}

vlbm_status vlbm_step_batch(vlbm_ctx* const* ctxs, int n_ctx, int64_t n_steps) {
    vlbm_status st = check_batch(ctxs, n_ctx);
    if (st) return st;
    if (n_steps < 0) return fail(VLBM_ERR_ARG, "n_steps < 0");
    return step_batch(ctxs, n_ctx, n_steps, ctxs[0]->stream);
}

vlbm_status vlbm_step_batch_persistent(vlbm_ctx* const* ctxs, int n_ctx, int64_t n_steps) {
    vlbm_status st = check_batch(ctxs, n_ctx);
    if (st) return st;
    if (n_steps < 0) return fail(VLBM_ERR_ARG, "n_steps < 0");
    return step_persistent(ctxs, n_ctx, n_steps, ctxs[0]->stream, false);
}

vlbm_status vlbm_set_barrier_spin_limit(uint32_t polls) {
    g_spin_limit = polls;
    return VLBM_OK;
}

namespace {
// Record n_steps of the contexts into a new graph; persistent: one persistent
// launch per 64 contexts, else the per-stage launches of vlbm_step_batch.
vlbm_status graph_record(vlbm_ctx* const* ctxs, int n_ctx, int64_t n_steps, bool persistent, vlbm_graph** out) {
    vlbm_status st = check_batch(ctxs, n_ctx);
    if (st) return st;
    if (!out || n_steps < 1) return fail(VLBM_ERR_ARG, "bad output pointer or n_steps < 1");
    vlbm_graph* g = new (std::nothrow) vlbm_graph();
    if (!g) return fail(VLBM_ERR_ALLOC, "host allocation failed");
    g->ctxs.assign(ctxs, ctxs + n_ctx);
    g->steps = n_steps;
    if (persistent)
        for (int c0 = 0; c0 < n_ctx; c0 += MAXRUNS) g->errs.push_back(at<uint32_t>(ctxs[c0], ctxs[c0]->L.bar) + 1);
    std::vector<int64_t> before(n_ctx);
    for (int i = 0; i < n_ctx; ++i) before[i] = ctxs[i]->launches;
    // capture on a private stream (the null stream cannot be captured); the
    // graph is launched later on the contexts' stream
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = persistent ? step_persistent(ctxs, n_ctx, n_steps, cs, true) : step_batch(ctxs, n_ctx, n_steps, cs);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (!st && e2 == hipSuccess) {
            e2 = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
            if (e2 == hipSuccess) g->graph = graph;
            else (void)hipGraphDestroy(graph);
        } else if (graph) {
            (void)hipGraphDestroy(graph);
        }
        e = e2;
    }
    if (cs) (void)hipStreamDestroy(cs);
    for (int i = 0; i < n_ctx; ++i) ctxs[i]->launches = before[i];
    if (st || e != hipSuccess) {
        delete g;
        return st ? st : fail(VLBM_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return VLBM_OK;
}
}  // namespace

vlbm_status vlbm_graph_create(vlbm_ctx* const* ctxs, int n_ctx, int64_t n_steps, vlbm_graph** out) {
    return graph_record(ctxs, n_ctx, n_steps, false, out);
}

vlbm_status vlbm_graph_create_persistent(vlbm_ctx* const* ctxs, int n_ctx, int64_t n_steps, vlbm_graph** out) {
    return graph_record(ctxs, n_ctx, n_steps, true, out);
}

vlbm_status vlbm_graph_check(vlbm_graph* g) {
    if (!g || !g->exec) return fail(VLBM_ERR_ARG, "bad graph");
    HIP_OK(hipStreamSynchronize(g->ctxs[0]->stream));
    for (const uint32_t* p : g->errs) {
        uint32_t err = 0;
        HIP_OK(hipMemcpy(&err, p, sizeof(err), hipMemcpyDeviceToHost));
        if (err)
            return fail(VLBM_ERR_DEVICE, "persistent graph: a grid barrier wait gave up; the runs' state is undefined");
    }
    return VLBM_OK;
}

vlbm_status vlbm_graph_launch(vlbm_graph* g) {
    if (!g || !g->exec) return fail(VLBM_ERR_ARG, "bad graph");
    HIP_OK(hipGraphLaunch(g->exec, g->ctxs[0]->stream));
    for (vlbm_ctx* x : g->ctxs) x->launches += 3 * g->steps;
    return VLBM_OK;
}

vlbm_status vlbm_graph_destroy(vlbm_graph* g) {
    if (!g) return VLBM_OK;
    delete g;
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

vlbm_status vlbm_correct_moments(vlbm_ctx* x, const double* drho, const double* dut,
                                 const double* dup, int on_dev) {
    if (!x || !drho || !dut || !dup) return fail(VLBM_ERR_ARG, "NULL argument");
    const int n = n_cells(x);
    double* F = at<double>(x, x->L.fields);
    const double *dr = drho, *da = dut, *db = dup;
    if (!on_dev) {
        HIP_OK(hipMemcpyAsync(F, drho, n * sizeof(double), hipMemcpyHostToDevice, x->stream));
        HIP_OK(hipMemcpyAsync(F + n, dut, n * sizeof(double), hipMemcpyHostToDevice, x->stream));
        HIP_OK(hipMemcpyAsync(F + 2 * (size_t)n, dup, n * sizeof(double), hipMemcpyHostToDevice, x->stream));
        dr = F; da = F + n; db = F + 2 * (size_t)n;
    }
    void* fn = x->ws + x->L.fbuf[0];
    vlbm_status st = dispatch(x->p.storage, [&](auto tag) {
        using St = decltype(tag);
        hipLaunchKernelGGL(correct_kernel<St>, dim3((n + 255) / 256), dim3(256), 0, x->stream,
                           fn, dr, da, db, x->c, n, x->p.rho0);
        return launch_check();
    });
    if (st) return st;
    if (!on_dev) HIP_OK(hipStreamSynchronize(x->stream));
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
                       at<double>(x, x->L.sgeo), dst, x->p.n_theta, x->p.n_phi, x->p.radius);
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
                           at<double>(x, x->L.sgeo), part, x->c, x->p.n_theta, x->p.n_phi,
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

// ---- diagnostics without a context or workspace -------------------------
// The scratch of vlbm_diagnostics_static: the per-block partial sums
// (RED_BLOCKS x 8 FP64) and the signed sin(theta) table of the grid
// (n_theta + 6 FP64).  One copy per device, held until the process ends;
// every call on a device shares it.
constexpr size_t STATIC_SCRATCH_DOUBLES = (size_t)1 << 17;              // 1 MiB
constexpr size_t STATIC_PART = 0, STATIC_SIN = (size_t)RED_BLOCKS * 8;
constexpr int STATIC_MAX_NTHETA = (int)(STATIC_SCRATCH_DOUBLES - STATIC_SIN) - 2 * NGH;
static __device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// The device address of this device's copy of the scratch array, looked up once
// per device (the array's name in host code is not a device address).
vlbm_status static_scratch(double** out) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(VLBM_ERR_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return VLBM_OK;
}

// signed sin(theta_j) for j = -3 .. nt + 2, the rows of the reduction's area
// element (the same expression as the context's host table)
__global__ void sin_rows_kernel(double* sinv, int nt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nt + 2 * NGH) sinv[j] = sin((j - NGH + 0.5) * (M_PI / nt));
}
}  // namespace

vlbm_status vlbm_diagnostics_static(int n_theta, int n_phi, int q, double radius, const double* f,
                                    double* out, void* hip_stream) {
    if (!f || !out) return fail(VLBM_ERR_ARG, "NULL argument");
    if (q != 3 && q != 4) return fail(VLBM_ERR_UNSUPPORTED, "q = %d: the quadratures are q = 3 and 4", q);
    if (n_theta < 1 || n_phi < 1 || !(radius > 0) || !std::isfinite(radius))
        return fail(VLBM_ERR_ARG, "bad grid or radius");
    if (n_theta > STATIC_MAX_NTHETA)
        return fail(VLBM_ERR_ARG, "n_theta = %d exceeds the static scratch (at most %d rows)", n_theta,
                    STATIC_MAX_NTHETA);
    if ((long long)n_theta * n_phi > (1LL << 31) - 1) return fail(VLBM_ERR_ARG, "grid too large");
    double* sc = nullptr;
    vlbm_status st = static_scratch(&sc);
    if (st) return st;
    Consts c;
    build_consts(c, VLBM_STORE_F64, q);
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int n = n_theta * n_phi;
    int nblk = (n + RED_T - 1) / RED_T;
    if (nblk > RED_BLOCKS) nblk = RED_BLOCKS;
    hipLaunchKernelGGL(sin_rows_kernel, dim3((n_theta + 2 * NGH + 255) / 256), dim3(256), 0, stream,
                       sc + STATIC_SIN, n_theta);
    if ((st = launch_check())) return st;
    // full populations: the deviation reference is 0
    hipLaunchKernelGGL(reduce_kernel<StF64>, dim3(nblk), dim3(RED_T), 0, stream, f, sc + STATIC_SIN,
                       sc + STATIC_PART, c, n_theta, n_phi, 0.0, radius);
    if ((st = launch_check())) return st;
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(64), 0, stream, sc + STATIC_PART, nblk, out);
    return launch_check();
}

// Host transfers go through the FP64 field staging area (4 planes) in chunks
// of four populations, so no device memory is allocated here.
vlbm_status vlbm_get_populations(vlbm_ctx* x, double* f, int on_dev) {
    if (!x || !f) return fail(VLBM_ERR_ARG, "NULL argument");
    const int n = n_cells(x);
    const void* fn = x->ws + x->L.fbuf[0];
    double* F = at<double>(x, x->L.fields);
    const int nk = x->p.q * x->p.q;
    for (int k0 = 0; k0 < nk; k0 += 4) {
        const int m = nk - k0 < 4 ? nk - k0 : 4;
        double* dst = on_dev ? f + (size_t)k0 * n : F;
        vlbm_status st = dispatch(x->p.storage, [&](auto tag) {
            using St = decltype(tag);
            hipLaunchKernelGGL(decode_kernel<St>, dim3((n + 255) / 256), dim3(256), 0, x->stream, fn,
                               dst, x->c, n, x->p.rho0, k0, m);
            return launch_check();
        });
        if (st) return st;
        if (!on_dev) {
            HIP_OK(hipMemcpyAsync(f + (size_t)k0 * n, F, m * (size_t)n * sizeof(double),
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
    const int nk = x->p.q * x->p.q;
    for (int k0 = 0; k0 < nk; k0 += 4) {
        const int m = nk - k0 < 4 ? nk - k0 : 4;
        const double* src = on_dev ? f + (size_t)k0 * n : F;
        if (!on_dev)
            HIP_OK(hipMemcpyAsync(F, f + (size_t)k0 * n, m * (size_t)n * sizeof(double),
                                  hipMemcpyHostToDevice, x->stream));
        vlbm_status st = dispatch(x->p.storage, [&](auto tag) {
            using St = decltype(tag);
            hipLaunchKernelGGL(encode_kernel<St>, dim3((n + 255) / 256), dim3(256), 0, x->stream, src,
                               fn, x->c, n, x->p.rho0, k0, m);
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

// closure.hip -- kernels of the learned-closure network (gfx950).
//
// A three-layer 3x3 CNN on the latitude-longitude grid corrects coarse vLBM
// moments.  The convolutions are implicit GEMMs on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation):
//   forward        D[pixel][co]  = sum_k  X_tap[pixel][k]   W[k][co]
//   data gradient  D[pixel][ci]  = sum_k  dZ_slot[pixel][k] W^T[k][ci]
//   weight grad.   D[co][ci]     = sum_px dZ[px][co]        X_tap[px][ci]   (per tap)
// A wavefront owns 16 pixels; one MFMA consumes K = 32.  Lane l of a wave
// supplies A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16], j = 0..7, and
// receives D[4 (l / 16) + i][l % 16], i = 0..3.
//
// Taps that leave the grid continue across a pole to phi + pi (the populations'
// ghost-row mapping, Sec. III.E); vector channels are negated there.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/vlbm_closure.h"

vlbm_status vlbm_set_error(vlbm_status st, const char* msg);   // vlbm.hip

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int WAVES = 4;            // wavefronts per block
constexpr int PIX_PER_BLOCK = 16 * WAVES;
constexpr int WCHUNK = 256;         // pixels per weight-gradient block

vlbm_status err(vlbm_status st, const char* fmt, ...) {
    char buf[400];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return vlbm_set_error(st, buf);
}

#define CLO_HIP(call)                                                                \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) return err(VLBM_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

vlbm_status launched() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return err(VLBM_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    return VLBM_OK;
}

__device__ __forceinline__ uint16_t to_bf16(float f) {
    // round to nearest even (finite inputs)
    const uint32_t b = __builtin_bit_cast(uint32_t, f);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}
__device__ __forceinline__ f32x4 mfma(u16x8 a, u16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

constexpr int kpad(int cin) { return (9 * cin + 31) / 32 * 32; }

// ---------------------------------------------------------------------------
// forward convolution
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_fwd_kernel(
    const uint16_t* __restrict__ x, const uint16_t* __restrict__ w, const float* __restrict__ bias,
    const int* __restrict__ nbr, const uint16_t* __restrict__ cross, uint32_t vmask, int HW,
    int P, int relu, float* __restrict__ z, uint16_t* __restrict__ a) {
    constexpr int K = 9 * CIN, KP = kpad(CIN), NB = COUT / 16;
    const int lane = threadIdx.x & 63;
    const int p0 = (blockIdx.x * WAVES + (threadIdx.x >> 6)) * 16;
    if (p0 >= P) return;
    const int m = lane & 15, g = lane >> 4;
    const int p = p0 + m;
    const int s = p / HW, hw = p - s * HW;
    const uint32_t cr = cross[hw];
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KP; kb += 32) {
        const int k0 = kb + 8 * g;              // 8 consecutive k share one tap (CIN % 8 == 0)
        u16x8 av = {0, 0, 0, 0, 0, 0, 0, 0};
        if (k0 < K) {
            const int t = k0 / CIN, ci0 = k0 - t * CIN;
            const int q = s * HW + nbr[hw * 9 + t];
            av = *reinterpret_cast<const u16x8*>(x + (size_t)q * CIN + ci0);
            if ((cr >> t) & 1u) {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if ((vmask >> (ci0 + j)) & 1u) av[j] ^= (uint16_t)0x8000u;
            }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const u16x8 bv = *reinterpret_cast<const u16x8*>(w + (size_t)(nb * 16 + m) * KP + k0);
            acc[nb] = mfma(av, bv, acc[nb]);
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + m;
        const float bc = bias[co];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const size_t o = (size_t)(p0 + 4 * g + i) * COUT + co;
            const float v = acc[nb][i] + bc;
            if (z) z[o] = v;
            a[o] = to_bf16(relu ? fmaxf(v, 0.f) : v);
        }
    }
}

// ---------------------------------------------------------------------------
// data gradient: cell q collects, in slot j, the tap of the cell inv[q][j]
// that reads q.  Interior rows: slot j is tap j.  The first row has no tap
// with dy = +1 reading it and instead two with dy = -1 (one across the pole):
// slots 6..8 hold those crossings with taps 0..2.  The last row mirrors this:
// slots 0..2 hold its crossings with taps 6..8.  16 pixels of a wave share a
// row (n_phi % 16 == 0), hence one tap per slot.
__device__ __forceinline__ int slot_tap(int slot, int row, int H) {
    if (row == 0 && slot >= 6) return slot - 6;
    if (row == H - 1 && slot < 3) return slot + 6;
    return slot;
}

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_bwd_data_kernel(
    const uint16_t* __restrict__ dz, const uint16_t* __restrict__ wt, const int* __restrict__ inv,
    int H, int W, int P, const float* __restrict__ zin, uint16_t* __restrict__ dx) {
    constexpr int K = 9 * COUT, KP = (K + 31) / 32 * 32, NB = CIN / 16;
    const int HW = H * W;
    const int lane = threadIdx.x & 63;
    const int p0 = (blockIdx.x * WAVES + (threadIdx.x >> 6)) * 16;
    if (p0 >= P) return;
    const int m = lane & 15, g = lane >> 4;
    const int q = p0 + m;
    const int s = q / HW, hw = q - s * HW;
    const int row = (p0 - s * HW) / W;          // the wave's row (uniform)
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KP; kb += 32) {
        const int k0 = kb + 8 * g;
        u16x8 av = {0, 0, 0, 0, 0, 0, 0, 0};
        int t = 0;
        const bool live = k0 < K;
        if (live) {
            const int slot = k0 / COUT, co0 = k0 - slot * COUT;
            const int src = s * HW + inv[hw * 9 + slot];
            av = *reinterpret_cast<const u16x8*>(dz + (size_t)src * COUT + co0);
            t = slot_tap(slot, row, H);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            u16x8 bv = {0, 0, 0, 0, 0, 0, 0, 0};
            if (live) {
                const int co0 = k0 % COUT;
                bv = *reinterpret_cast<const u16x8*>(wt + ((size_t)t * CIN + nb * 16 + m) * COUT + co0);
            }
            acc[nb] = mfma(av, bv, acc[nb]);
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int ci = nb * 16 + m;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const size_t o = (size_t)(p0 + 4 * g + i) * CIN + ci;
            dx[o] = to_bf16(zin[o] > 0.f ? acc[nb][i] : 0.f);
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: block (chunk, tap) covers WSUB x WCHUNK pixels; for each
// WCHUNK of them it stages dZ and the tap-gathered input in LDS and the matrix
// cores accumulate their product over the pixels in registers.  A second
// kernel sums the chunks' partials in a fixed order (deterministic).
constexpr int WSUB = 4;                 // WCHUNK slices per weight-gradient block
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_bwd_w_kernel(
    const uint16_t* __restrict__ x, const uint16_t* __restrict__ dz, const int* __restrict__ nbr,
    const uint16_t* __restrict__ cross, uint32_t vmask, int HW, int P, float* __restrict__ part,
    float* __restrict__ partb) {
    constexpr int CI16 = CIN < 16 ? 16 : CIN;   // B operand columns
    constexpr int XS = CI16 + 2, DS = COUT + 2; // LDS row strides (odd dword count)
    __shared__ uint16_t xs[WCHUNK * XS];
    __shared__ uint16_t ds[WCHUNK * DS];
    const int chunk = blockIdx.x, t = blockIdx.y, tid = threadIdx.x;
    constexpr int MB = COUT / 16, NBc = CI16 / 16;
    constexpr int NPAIR = (MB * NBc + WAVES - 1) / WAVES;    // (mb, nb) pairs per wave
    const int wv = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
    f32x4 acc[NPAIR];
#pragma unroll
    for (int j = 0; j < NPAIR; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float sb = 0.f;                            // bias gradient (tap 4, threads < COUT)
    for (int sub = 0; sub < WSUB; ++sub) {
        const int p = (chunk * WSUB + sub) * WCHUNK + tid;
        if (p < P) {
            const int s = p / HW, hw = p - s * HW;
            const int q = s * HW + nbr[hw * 9 + t];
            const bool flip = (cross[hw] >> t) & 1u;
#pragma unroll
            for (int ci = 0; ci < CI16; ++ci) {
                uint16_t v = ci < CIN ? x[(size_t)q * CIN + ci] : (uint16_t)0;
                if (flip && ci < CIN && ((vmask >> ci) & 1u)) v ^= (uint16_t)0x8000u;
                xs[tid * XS + ci] = v;
            }
#pragma unroll
            for (int co = 0; co < COUT; ++co) ds[tid * DS + co] = dz[(size_t)p * COUT + co];
        } else {
            for (int ci = 0; ci < CI16; ++ci) xs[tid * XS + ci] = 0;
            for (int co = 0; co < COUT; ++co) ds[tid * DS + co] = 0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NPAIR; ++j) {
            const int pair = wv + WAVES * j;
            if (pair < MB * NBc) {
                const int mb = pair / NBc, nb = pair % NBc;
                for (int kb = 0; kb < WCHUNK; kb += 32) {
                    u16x8 av, bv;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int px = kb + 8 * g + i;
                        av[i] = ds[px * DS + mb * 16 + m];
                        bv[i] = xs[px * XS + nb * 16 + m];
                    }
                    acc[j] = mfma(av, bv, acc[j]);
                }
            }
        }
        if (t == 4 && tid < COUT)
            for (int i = 0; i < WCHUNK; ++i) sb += from_bf16(ds[i * DS + tid]);
        __syncthreads();                       // the slices are overwritten next
    }
#pragma unroll
    for (int j = 0; j < NPAIR; ++j) {
        const int pair = wv + WAVES * j;
        if (pair < MB * NBc) {
            const int mb = pair / NBc, nb = pair % NBc;
            const int ci = nb * 16 + m;
            if (ci < CIN) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int co = mb * 16 + 4 * g + i;
                    part[(((size_t)chunk * 9 + t) * COUT + co) * CIN + ci] = acc[j][i];
                }
            }
        }
    }
    if (t == 4 && tid < COUT) partb[(size_t)chunk * COUT + tid] = sb;
}

// Sum of the chunks' partials, in a fixed order: block b takes 64 consecutive
// partial entries (weights in the partials' order, then the biases); wave w
// adds chunks w, w + 16, w + 32, ... in turn, and the 16 wave sums are added in
// wave order.
constexpr int RW_WAVES = 16;
__global__ __launch_bounds__(64 * RW_WAVES) void reduce_w_kernel(
    const float* __restrict__ part, const float* __restrict__ partb, int nchunk, int cin, int cout,
    float* __restrict__ dw, float* __restrict__ db) {
    __shared__ float sh[RW_WAVES][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = cout * 9 * cin;
    const int e = blockIdx.x * 64 + lane;       // entry: weight (partials' order) or bias
    float s = 0.f;
    if (e < nw) {
        for (int c = wv; c < nchunk; c += RW_WAVES) s += part[(size_t)c * nw + e];
    } else if (e < nw + cout) {
        for (int c = wv; c < nchunk; c += RW_WAVES) s += partb[(size_t)c * cout + (e - nw)];
    }
    sh[wv][lane] = s;
    __syncthreads();
    if (wv == 0) {
        float tot = sh[0][lane];
        for (int w = 1; w < RW_WAVES; ++w) tot += sh[w][lane];
        if (e < nw) {
            // partial order (t, co, ci) -> weight order (co, t, ci)
            const int t = e / (cout * cin), r = e - t * cout * cin, co = r / cin, ci = r - co * cin;
            dw[(size_t)co * 9 * cin + t * cin + ci] = tot;
        } else if (e < nw + cout) {
            db[e - nw] = tot;
        }
    }
}

// ---------------------------------------------------------------------------
// loss, optimiser, packing
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ z,
                                                   const float* __restrict__ tgt, int H, int W,
                                                   int P, float inv_norm, uint16_t* __restrict__ dz,
                                                   float* __restrict__ part) {
    __shared__ float red[256];
    const int p = blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (p < P) {
        const int r = (p % (H * W)) / W;
        const float w = (float)sin((r + 0.5) * M_PI / H);
        for (int c = 0; c < 16; ++c) {
            float gz = 0.f;
            if (c < 3) {
                const float d = z[(size_t)p * 16 + c] - tgt[(size_t)p * 3 + c];
                l += w * d * d;
                gz = 2.f * w * d * inv_norm;
            }
            dz[(size_t)p * 16 + c] = to_bf16(gz);
        }
    }
    red[threadIdx.x] = l * inv_norm;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void adam_kernel(int n, float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, float c1, float c2,
                            float lr, float b1, float b2, float eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void pack_w_kernel(const float* __restrict__ master, int cin, int cout, int kp,
                              uint16_t* __restrict__ w, uint16_t* __restrict__ wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cout * kp) return;
    const int co = i / kp, k = i - co * kp;
    const uint16_t h = k < 9 * cin ? to_bf16(master[co * 9 * cin + k]) : (uint16_t)0;
    w[i] = h;
    if (k < 9 * cin) {
        const int t = k / cin, ci = k - t * cin;
        wt[((size_t)t * cin + ci) * cout + co] = h;
    }
}

__global__ void pack_input_kernel(int P, const double* __restrict__ rho,
                                  const double* __restrict__ ut, const double* __restrict__ up,
                                  const double* __restrict__ T, double s_rho, double s_u,
                                  double s_T, uint16_t* __restrict__ x) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    v[0] = to_bf16((float)((rho[p] - 1.0) * s_rho));
    v[1] = to_bf16((float)(ut[p] * s_u));
    v[2] = to_bf16((float)(up[p] * s_u));
    if (T) v[3] = to_bf16((float)((T[p] - 1.0) * s_T));
    *reinterpret_cast<u16x8*>(x + (size_t)p * 8) = v;
}

__global__ void unpack_output_kernel(int P, const float* __restrict__ z, double o_rho, double o_u,
                                     double* __restrict__ dr, double* __restrict__ dut,
                                     double* __restrict__ dup) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    dr[p] = (double)z[(size_t)p * 16] * o_rho;
    dut[p] = (double)z[(size_t)p * 16 + 1] * o_u;
    dup[p] = (double)z[(size_t)p * 16 + 2] * o_u;
}

__global__ void pack_target_kernel(int P, const double* __restrict__ ra, const double* __restrict__ ua,
                                   const double* __restrict__ va, const double* __restrict__ rb,
                                   const double* __restrict__ ub, const double* __restrict__ vb,
                                   double i_rho, double i_u, float* __restrict__ t) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    t[(size_t)p * 3] = (float)((ra[p] - rb[p]) * i_rho);
    t[(size_t)p * 3 + 1] = (float)((ua[p] - ub[p]) * i_u);
    t[(size_t)p * 3 + 2] = (float)((va[p] - vb[p]) * i_u);
}

__global__ void box_filter_kernel(int Hf, int Wf, int f, int n, const double* __restrict__ rho,
                                  const double* __restrict__ ut, const double* __restrict__ up,
                                  double* __restrict__ rc, double* __restrict__ uc,
                                  double* __restrict__ vc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int Hc = Hf / f, Wc = Wf / f;
    if (i >= n) return;
    const int b = i / (Hc * Wc), rr = (i / Wc) % Hc, cc = i % Wc;
    double ws = 0, m = 0, mu = 0, mv = 0;
    for (int a = 0; a < f; ++a) {
        const int r = rr * f + a;
        const double w = sin((r + 0.5) * M_PI / Hf);
        for (int c = 0; c < f; ++c) {
            const size_t o = ((size_t)b * Hf + r) * Wf + cc * f + c;
            ws += w;
            m += w * rho[o];
            mu += w * rho[o] * ut[o];
            mv += w * rho[o] * up[o];
        }
    }
    rc[i] = m / ws;
    uc[i] = mu / m;
    vc[i] = mv / m;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct CloLayout {
    size_t nbr, cross, inv, part, partb, lpart, total;
    int nchunk, nlblk;
};

CloLayout clo_layout(int H, int W, int B) {
    CloLayout L{};
    const size_t HW = (size_t)H * W, P = HW * B;
    L.nchunk = (int)((P + WCHUNK - 1) / WCHUNK);
    L.nlblk = (int)((P + 255) / 256);
    size_t off = 0;
    L.nbr = off; off += align256(HW * 9 * sizeof(int));
    L.cross = off; off += align256(HW * sizeof(uint16_t));
    L.inv = off; off += align256(HW * 9 * sizeof(int));
    L.part = off; off += align256((size_t)L.nchunk * 9 * 32 * 32 * sizeof(float));
    L.partb = off; off += align256((size_t)L.nchunk * 32 * sizeof(float));
    L.lpart = off; off += align256((size_t)L.nlblk * sizeof(float));
    L.total = off;
    return L;
}

bool grid_ok(int H, int W, int B) {
    return H >= 2 && W >= 16 && W % 16 == 0 && B >= 1 && (double)H * W * B < 2e9;
}

}  // namespace

struct vlbm_clo {
    int H, W, max_batch;
    hipStream_t stream;
    char* ws;
    CloLayout L;
};

namespace {

bool shape_ok(int cin, int cout) { return (cin == 8 || cin == 32) && (cout == 16 || cout == 32); }

vlbm_status check_batch(const vlbm_clo* c, int batch) {
    if (!c) return err(VLBM_ERR_ARG, "NULL closure context");
    if (batch < 1 || batch > c->max_batch)
        return err(VLBM_ERR_ARG, "batch %d outside 1..%d", batch, c->max_batch);
    return VLBM_OK;
}

template <class F>
vlbm_status by_shape(int cin, int cout, F&& f) {
    if (cin == 8 && cout == 32) return f(std::integral_constant<int, 8>{}, std::integral_constant<int, 32>{});
    if (cin == 32 && cout == 32) return f(std::integral_constant<int, 32>{}, std::integral_constant<int, 32>{});
    if (cin == 32 && cout == 16) return f(std::integral_constant<int, 32>{}, std::integral_constant<int, 16>{});
    if (cin == 8 && cout == 16) return f(std::integral_constant<int, 8>{}, std::integral_constant<int, 16>{});
    return err(VLBM_ERR_ARG, "layer shape %d -> %d not supported (cin 8|32, cout 16|32)", cin, cout);
}

}  // namespace

extern "C" {

size_t vlbm_clo_workspace_bytes(int n_theta, int n_phi, int max_batch) {
    if (!grid_ok(n_theta, n_phi, max_batch)) return 0;
    return clo_layout(n_theta, n_phi, max_batch).total;
}

vlbm_status vlbm_clo_create(int H, int W, int B, void* stream, void* workspace, size_t bytes,
                            vlbm_clo** out) {
    if (!out || !workspace) return err(VLBM_ERR_ARG, "NULL output or workspace");
    *out = nullptr;
    if (!grid_ok(H, W, B))
        return err(VLBM_ERR_ARG, "grid %dx%d batch %d: need n_theta >= 2, n_phi a multiple of 16", H, W, B);
    const CloLayout L = clo_layout(H, W, B);
    if (bytes < L.total) return err(VLBM_ERR_ALLOC, "workspace %zu bytes < %zu", bytes, L.total);
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return err(VLBM_ERR_ARG, "workspace not 256-byte aligned");
    // tap tables: nbr (cell read by each tap), cross (taps across a pole), inv
    // (cells whose taps read a cell, by slot; see slot_tap)
    const int HW = H * W;
    std::vector<int> nbr((size_t)HW * 9), inv((size_t)HW * 9, -1);
    std::vector<uint16_t> cross(HW, 0);
    for (int r = 0; r < H; ++r)
        for (int cc = 0; cc < W; ++cc)
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3 - 1, dx = t % 3 - 1;
                int rr = r + dy, c2 = cc + dx;
                bool x = false;
                if (rr < 0) { rr = -rr - 1; c2 += W / 2; x = true; }
                else if (rr >= H) { rr = 2 * H - rr - 1; c2 += W / 2; x = true; }
                c2 = ((c2 % W) + W) % W;
                nbr[(size_t)(r * W + cc) * 9 + t] = rr * W + c2;
                if (x) cross[r * W + cc] |= (uint16_t)(1u << t);
            }
    for (int r = 0; r < H; ++r)
        for (int cc = 0; cc < W; ++cc)
            for (int j = 0; j < 9; ++j) {
                const int dy = j / 3 - 1, dx = j % 3 - 1;
                int pr, pc;
                if (r == 0 && j >= 6) { pr = 0; pc = cc - dx - W / 2; }
                else if (r == H - 1 && j < 3) { pr = H - 1; pc = cc - dx - W / 2; }
                else { pr = r - dy; pc = cc - dx; }
                pc = ((pc % W) + W) % W;
                inv[(size_t)(r * W + cc) * 9 + j] = pr * W + pc;
            }
    // self-check: slot j of cell q is read by tap slot_tap(j) of inv[q][j]
    for (int q = 0; q < HW; ++q)
        for (int j = 0; j < 9; ++j) {
            const int r = q / W;
            int t = j;
            if (r == 0 && j >= 6) t = j - 6;
            else if (r == H - 1 && j < 3) t = j + 6;
            const int p = inv[(size_t)q * 9 + j];
            if (p < 0 || p >= HW || nbr[(size_t)p * 9 + t] != q)
                return err(VLBM_ERR_ARG, "internal: inverse tap table inconsistent at cell %d slot %d", q, j);
        }
    vlbm_clo* c = new (std::nothrow) vlbm_clo;
    if (!c) return err(VLBM_ERR_ALLOC, "host allocation failed");
    c->H = H; c->W = W; c->max_batch = B;
    c->stream = static_cast<hipStream_t>(stream);
    c->ws = static_cast<char*>(workspace);
    c->L = L;
    hipError_t e = hipMemcpyAsync(c->ws + L.nbr, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + L.cross, cross.data(), cross.size() * sizeof(uint16_t), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + L.inv, inv.data(), inv.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return err(VLBM_ERR_DEVICE, "uploading tap tables: %s", hipGetErrorString(e));
    }
    *out = c;
    return VLBM_OK;
}

vlbm_status vlbm_clo_destroy(vlbm_clo* c) {
    delete c;
    return VLBM_OK;
}

vlbm_status vlbm_clo_conv_forward(vlbm_clo* c, int cin, int cout, int batch, const void* x,
                                  const void* w, const float* bias, uint32_t vmask, int relu,
                                  float* z, void* a) {
    if (vlbm_status st = check_batch(c, batch)) return st;
    if (!x || !w || !bias || !a) return err(VLBM_ERR_ARG, "NULL tensor");
    if (!shape_ok(cin, cout)) return err(VLBM_ERR_ARG, "layer shape %d -> %d", cin, cout);
    const int HW = c->H * c->W, P = HW * batch;
    return by_shape(cin, cout, [&](auto ci, auto co) {
        hipLaunchKernelGGL((conv_fwd_kernel<decltype(ci)::value, decltype(co)::value>),
                           dim3((P + PIX_PER_BLOCK - 1) / PIX_PER_BLOCK), dim3(256), 0, c->stream,
                           static_cast<const uint16_t*>(x), static_cast<const uint16_t*>(w), bias,
                           reinterpret_cast<const int*>(c->ws + c->L.nbr),
                           reinterpret_cast<const uint16_t*>(c->ws + c->L.cross), vmask, HW, P,
                           relu, z, static_cast<uint16_t*>(a));
        return launched();
    });
}

vlbm_status vlbm_clo_conv_backward_data(vlbm_clo* c, int cin, int cout, int batch, const void* dz,
                                        const void* wt, const float* zin, void* dx) {
    if (vlbm_status st = check_batch(c, batch)) return st;
    if (!dz || !wt || !zin || !dx) return err(VLBM_ERR_ARG, "NULL tensor");
    if (cin != 32 || (cout != 16 && cout != 32))
        return err(VLBM_ERR_ARG, "data gradient needs a 32-channel hidden input (cin %d, cout %d)", cin, cout);
    const int P = c->H * c->W * batch;
    auto go = [&](auto co) {
        hipLaunchKernelGGL((conv_bwd_data_kernel<32, decltype(co)::value>),
                           dim3((P + PIX_PER_BLOCK - 1) / PIX_PER_BLOCK), dim3(256), 0, c->stream,
                           static_cast<const uint16_t*>(dz), static_cast<const uint16_t*>(wt),
                           reinterpret_cast<const int*>(c->ws + c->L.inv), c->H, c->W, P, zin,
                           static_cast<uint16_t*>(dx));
        return launched();
    };
    return cout == 32 ? go(std::integral_constant<int, 32>{}) : go(std::integral_constant<int, 16>{});
}

vlbm_status vlbm_clo_conv_backward_weight(vlbm_clo* c, int cin, int cout, int batch, const void* x,
                                          const void* dz, uint32_t vmask, float* dw, float* db) {
    if (vlbm_status st = check_batch(c, batch)) return st;
    if (!x || !dz || !dw || !db) return err(VLBM_ERR_ARG, "NULL tensor");
    if (!shape_ok(cin, cout)) return err(VLBM_ERR_ARG, "layer shape %d -> %d", cin, cout);
    const int HW = c->H * c->W, P = HW * batch;
    const int nchunk = (P + WSUB * WCHUNK - 1) / (WSUB * WCHUNK);
    float* part = reinterpret_cast<float*>(c->ws + c->L.part);
    float* partb = reinterpret_cast<float*>(c->ws + c->L.partb);
    vlbm_status st = by_shape(cin, cout, [&](auto ci, auto co) {
        hipLaunchKernelGGL((conv_bwd_w_kernel<decltype(ci)::value, decltype(co)::value>),
                           dim3(nchunk, 9), dim3(256), 0, c->stream,
                           static_cast<const uint16_t*>(x), static_cast<const uint16_t*>(dz),
                           reinterpret_cast<const int*>(c->ws + c->L.nbr),
                           reinterpret_cast<const uint16_t*>(c->ws + c->L.cross), vmask, HW, P,
                           part, partb);
        return launched();
    });
    if (st) return st;
    const int n = cout * 9 * cin + cout;
    hipLaunchKernelGGL(reduce_w_kernel, dim3((n + 63) / 64), dim3(64 * RW_WAVES), 0, c->stream, part,
                       partb, nchunk, cin, cout, dw, db);
    return launched();
}

vlbm_status vlbm_clo_loss(vlbm_clo* c, int batch, const float* z, const float* target, void* dz,
                          float* partials, int* n_partials) {
    if (vlbm_status st = check_batch(c, batch)) return st;
    if (!z || !target || !dz || !partials || !n_partials) return err(VLBM_ERR_ARG, "NULL tensor");
    const int P = c->H * c->W * batch;
    double wsum = 0;
    for (int r = 0; r < c->H; ++r) wsum += std::sin((r + 0.5) * M_PI / c->H);
    const float inv_norm = (float)(1.0 / (3.0 * batch * c->W * wsum));
    const int nb = (P + 255) / 256;
    hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(256), 0, c->stream, z, target, c->H, c->W, P,
                       inv_norm, static_cast<uint16_t*>(dz), partials);
    *n_partials = nb;
    return launched();
}

vlbm_status vlbm_clo_adam(vlbm_clo* c, int n, float* p, const float* g, float* m, float* v,
                          int step, float lr, float b1, float b2, float eps) {
    if (!c || !p || !g || !m || !v || n < 0 || step < 1) return err(VLBM_ERR_ARG, "bad Adam arguments");
    if (n == 0) return VLBM_OK;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, step)));
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, n, p, g, m, v,
                       c1, c2, lr, b1, b2, eps);
    return launched();
}

vlbm_status vlbm_clo_pack_weights(vlbm_clo* c, int cin, int cout, const float* master, void* w,
                                  void* wt) {
    if (!c || !master || !w || !wt) return err(VLBM_ERR_ARG, "NULL tensor");
    if (!shape_ok(cin, cout)) return err(VLBM_ERR_ARG, "layer shape %d -> %d", cin, cout);
    const int kp = kpad(cin), n = cout * kp;
    hipLaunchKernelGGL(pack_w_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, master, cin,
                       cout, kp, static_cast<uint16_t*>(w), static_cast<uint16_t*>(wt));
    return launched();
}

vlbm_status vlbm_clo_pack_input(vlbm_clo* c, int batch, const double* rho, const double* ut,
                                const double* up, const double* T, double s_rho, double s_u,
                                double s_T, void* x) {
    if (vlbm_status st = check_batch(c, batch)) return st;
    if (!rho || !ut || !up || !x) return err(VLBM_ERR_ARG, "NULL tensor");
    const int P = c->H * c->W * batch;
    hipLaunchKernelGGL(pack_input_kernel, dim3((P + 255) / 256), dim3(256), 0, c->stream, P, rho,
                       ut, up, T, s_rho, s_u, s_T, static_cast<uint16_t*>(x));
    return launched();
}

vlbm_status vlbm_clo_unpack_output(vlbm_clo* c, int batch, const float* z, double o_rho,
                                   double o_u, double* dr, double* dut, double* dup) {
    if (vlbm_status st = check_batch(c, batch)) return st;
    if (!z || !dr || !dut || !dup) return err(VLBM_ERR_ARG, "NULL tensor");
    const int P = c->H * c->W * batch;
    hipLaunchKernelGGL(unpack_output_kernel, dim3((P + 255) / 256), dim3(256), 0, c->stream, P, z,
                       o_rho, o_u, dr, dut, dup);
    return launched();
}

vlbm_status vlbm_clo_pack_target(vlbm_clo* c, int batch, const double* ra, const double* ua,
                                 const double* va, const double* rb, const double* ub,
                                 const double* vb, double o_rho, double o_u, float* t) {
    if (vlbm_status st = check_batch(c, batch)) return st;
    if (!ra || !ua || !va || !rb || !ub || !vb || !t) return err(VLBM_ERR_ARG, "NULL tensor");
    if (!(o_rho > 0) || !(o_u > 0)) return err(VLBM_ERR_ARG, "output scales must be > 0");
    const int P = c->H * c->W * batch;
    hipLaunchKernelGGL(pack_target_kernel, dim3((P + 255) / 256), dim3(256), 0, c->stream, P, ra, ua,
                       va, rb, ub, vb, 1.0 / o_rho, 1.0 / o_u, t);
    return launched();
}

vlbm_status vlbm_box_filter(int Hf, int Wf, int f, int batch, const double* rho, const double* ut,
                            const double* up, double* rc, double* uc, double* vc, void* stream) {
    if (f < 1 || Hf < f || Wf < f || Hf % f || Wf % f || batch < 1)
        return err(VLBM_ERR_ARG, "box filter: %dx%d by %d (batch %d)", Hf, Wf, f, batch);
    if (!rho || !ut || !up || !rc || !uc || !vc) return err(VLBM_ERR_ARG, "NULL field");
    const int n = (Hf / f) * (Wf / f) * batch;
    hipLaunchKernelGGL(box_filter_kernel, dim3((n + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), Hf, Wf, f, n, rho, ut, up, rc, uc, vc);
    return launched();
}

}  // extern "C"

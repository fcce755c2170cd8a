// sc_pinn.hip -- the PINN surrogate of Li & Zhang (arXiv 2504.10539) on the
// GPU: the network of Sec. III-B evaluated at every cell (Eq. (2),
// lbm_pinn_infer), and the Sec. II-C correction of a run's state at its
// interface cells (Eq. (9) criterion, Eq. (16) gradient; lbm_pinn_correct).
//
// The network maps the cell centre scaled to (-1, 1) to (rho, u_x, u_y)
// through hidden layers of 64, 128, 128 and 64 tanh neurons and a linear
// output layer.  Layers 2 to 4 are dense contractions over a tile of 64 cells
// and run on the matrix cores: v_mfma_f32_16x16x16f16 with FP16 weights and
// activations and FP32 accumulation.  Each wavefront of a workgroup owns a
// slice of every layer's output features and keeps that slice's weights in
// registers for the whole launch; activations pass between layers through
// LDS in FP16.  Layer 1 (two inputs) and layer 5 (three outputs) are FP32
// FMAs, tanh is the FP32 libm function.
//
// The correction works on the interface cells only: tiles without one are
// skipped after the Eq. (16) test (FP64 density, as the diagnostics compute
// it).  On an interface cell, with rho and u = sum_i f_i e_i / rho of its
// pulled populations and the network's rho_N, u_N:
//   rho' = rho + beta (rho_N - rho),  u' = u + beta (u_N - u),
//   f_i <- f_i + f_eq_i(rho', u') - f_eq_i(rho, u),
// written back to the stored values the cell pulls, so that the
// non-equilibrium part is kept and the cell carries exactly rho' and rho' u'.
#include <hip/hip_runtime.h>

#include "sc_runtime.h"

namespace sclbm {
namespace {

// Sec. III-B layer widths and the offsets of each layer in the packed FP32
// parameter vector (W_l row-major as (out, in), then b_l; layer order).
constexpr int kH1 = 64, kH2 = 128, kH3 = 128, kH4 = 64, kOut = 3;
constexpr int oW1 = 0, oB1 = oW1 + kH1 * 2, oW2 = oB1 + kH1, oB2 = oW2 + kH2 * kH1,
              oW3 = oB2 + kH2, oB3 = oW3 + kH3 * kH2, oW4 = oB3 + kH3, oB4 = oW4 + kH4 * kH3,
              oW5 = oB4 + kH4, oB5 = oW5 + kOut * kH4, kParams = oB5 + kOut;
static_assert(kParams == LBM_PINN_PARAMS, "parameter layout");

constexpr int kTile = 64;            // cells per tile: one row segment, one cell per lane
constexpr int kThreads = 256;        // four wavefronts
constexpr int kStride = kH2 + 8;     // LDS row stride of the activations (halves)
constexpr double kInterface = 0.01;  // Eq. (9) threshold on |grad rho|

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

// tanh(z) = 1 - 2 / (exp(2 z) + 1) from the hardware base-2 exponential and
// reciprocal: five instructions where the library tanhf takes some thirty.
// The form holds for either sign (exp(2 z) = inf gives 1, exp(2 z) = 0 gives
// -1).  Its absolute error stays below 4e-7 (every float z with
// 2^-30 <= |z| <= 20 checked against FP64 tanh), far below the
// half-precision rounding of the activation that follows.
__device__ __forceinline__ float tanh_fast(float z) {
  const float e = __builtin_amdgcn_exp2f(z * 2.88539004f);  // 2 log2(e)
  return fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

// One 16 x 16 x 16 matrix multiply-add on the matrix cores.  Lane l holds
// A[l % 16][4 (l / 16) + j], B[4 (l / 16) + j][l % 16] (j = 0..3, one half
// each) and D[4 (l / 16) + j][l % 16] (one float each).
__device__ __forceinline__ float4v mfma16(half4 a, half4 b, float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// A fragments of one layer for the wavefront's output features: feature
// m = col0 + 16 cb + (lane % 16), inputs k = 16 s + 4 (lane / 16) + j, from
// W (out x in, FP32) rounded to half.
template <int KS, int NCB>
__device__ __forceinline__ void load_weights(const float* __restrict__ W, int in, int col0,
                                             int lane, half4 (&w)[NCB][KS]) {
  const int nl = lane & 15, kq = 4 * (lane >> 4);
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        w[cb][s][j] = static_cast<_Float16>(W[(size_t)(col0 + 16 * cb + nl) * in + 16 * s + kq + j]);
}

// One hidden layer over the tile's 64 cells: out = tanh(W in + b) for the
// wavefront's features col0 .. col0 + 16 NCB - 1, with KS blocks of 16 inputs.
// The weights are the A operand and the activations (cells as columns) the B
// operand, so each lane's four results are four consecutive features of one
// cell: they go to LDS as one 8-byte write, and the accumulators start from
// the biases.
template <int KS, int NCB>
__device__ __forceinline__ void dense_tanh(const _Float16 (*in)[kStride], _Float16 (*out)[kStride],
                                           const half4 (&w)[NCB][KS], const float* bias, int col0,
                                           int lane) {
  const int r16 = lane & 15, kq = 4 * (lane >> 4);
  float4v b[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) b[cb] = *reinterpret_cast<const float4v*>(&bias[col0 + 16 * cb + kq]);
#pragma unroll
  for (int rb = 0; rb < kTile / 16; ++rb) {
    float4v acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = b[cb];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const half4 a = *reinterpret_cast<const half4*>(&in[rb * 16 + r16][16 * s + kq]);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma16(w[cb][s], a, acc[cb]);
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      half4 h;
#pragma unroll
      for (int j = 0; j < 4; ++j) h[j] = static_cast<_Float16>(tanh_fast(acc[cb][j]));
      *reinterpret_cast<half4*>(&out[rb * 16 + r16][col0 + 16 * cb + kq]) = h;
    }
  }
}

// Second-order equilibrium in FP32: w_i rho (1 + 3 e_i.u + 4.5 (e_i.u)^2 - 1.5 u.u).
__device__ __forceinline__ void equilibrium32(float rho, float ux, float uy, float (&e)[9]) {
  const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
  const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const float usq = fmaf(ux, ux, uy * uy);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float eu = (float)ex[i] * ux + (float)ey[i] * uy;
    const float poly = fmaf(4.5f * eu, eu, fmaf(3.0f, eu, fmaf(-1.5f, usq, 1.0f)));
    e[i] = ws[i] * rho * poly;
  }
}

struct PinnArgs {
  void* pop;            // the run's current population buffer
  const double* rho64;  // FP64 density of that state (correction only)
  const float* params;  // packed FP32 network parameters
  float* out[3];        // inference: rho_N, u_x, u_y planes (each may be null)
  uint8_t* mask;        // correction: 1 where a cell was corrected, 0 elsewhere (may be null)
  int nx, ny;
  float rho0;           // FP16-shifted storage's shift density
  float beta;           // correction: blending factor
};

// CORRECT = false: the network's fields at every cell into out[].  CORRECT =
// true: the interface correction of the state in place.
template <class S, bool CORRECT>
__global__ __launch_bounds__(kThreads) void k_pinn(PinnArgs a) {
  using T = typename S::T;
  __shared__ __attribute__((aligned(16))) _Float16 act[2][kTile][kStride];
  __shared__ float part[kThreads / 64][kOut][kTile];  // layer-5 partial sums per wavefront
  __shared__ float sw1[kH1][2], sb1[kH1], sw5[kOut][kH4], sb5[kOut];
  __shared__ __attribute__((aligned(16))) float sb2[kH2], sb3[kH3], sb4[kH4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float* P = a.params;
  for (int i = threadIdx.x; i < kH1; i += kThreads) {
    sw1[i][0] = P[oW1 + 2 * i];
    sw1[i][1] = P[oW1 + 2 * i + 1];
    sb1[i] = P[oB1 + i];
    sb4[i] = P[oB4 + i];
  }
  for (int i = threadIdx.x; i < kH2; i += kThreads) {
    sb2[i] = P[oB2 + i];
    sb3[i] = P[oB3 + i];
  }
  for (int i = threadIdx.x; i < kOut * kH4; i += kThreads) sw5[i / kH4][i % kH4] = P[oW5 + i];
  if (threadIdx.x < kOut) sb5[threadIdx.x] = P[oB5 + threadIdx.x];
  // this wavefront's weight slices: layers 2 and 3 output features
  // 32 w .. 32 w + 31, layer 4 features 16 w .. 16 w + 15
  half4 w2[2][kH1 / 16], w3[2][kH2 / 16], w4[1][kH3 / 16];
  load_weights(P + oW2, kH1, 32 * wave, lane, w2);
  load_weights(P + oW3, kH2, 32 * wave, lane, w3);
  load_weights(P + oW4, kH3, 16 * wave, lane, w4);
  __syncthreads();

  const int nx = a.nx, ny = a.ny;
  const int tiles_x = (nx + kTile - 1) / kTile;
  const int ntiles = tiles_x * ny;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int y = t / tiles_x, x = (t % tiles_x) * kTile + lane;
    const bool live = x < nx;
    bool m = false;
    if constexpr (CORRECT) {
      // Eq. (9) criterion with the Eq. (16) gradient (periodic), in FP64
      if (live) {
        const double* r = a.rho64;
        const size_t r0 = (size_t)y * nx;
        const double gx = (r[r0 + wrap_inc(x, nx)] - r[r0 + wrap_dec(x, nx)]) / 2.0;
        const double gy = (r[(size_t)wrap_inc(y, ny) * nx + x] - r[(size_t)wrap_dec(y, ny) * nx + x]) / 2.0;
        m = sqrt(gx * gx + gy * gy) > kInterface;
      }
      if (wave == 0 && live && a.mask) a.mask[(size_t)y * nx + x] = m ? 1 : 0;
      // every wavefront finds the same cells, so the whole workgroup skips
      if (__builtin_amdgcn_ballot_w64(m) == 0) continue;
    }
    // layer 1 (FP32): this wavefront's 16 features of the lane's cell
    {
      const float xh = (float)(2 * x + 1) / (float)nx - 1.0f;
      const float yh = (float)(2 * y + 1) / (float)ny - 1.0f;
      typedef _Float16 half8 __attribute__((ext_vector_type(8)));
      half8 h[2];
#pragma unroll
      for (int f = 0; f < 16; ++f) {
        const int n = 16 * wave + f;
        const float z = fmaf(sw1[n][0], xh, fmaf(sw1[n][1], yh, sb1[n]));
        h[f / 8][f % 8] = static_cast<_Float16>(tanh_fast(z));
      }
      half8* dst = reinterpret_cast<half8*>(&act[0][lane][16 * wave]);
      dst[0] = h[0];
      dst[1] = h[1];
    }
    __syncthreads();
    dense_tanh(act[0], act[1], w2, sb2, 32 * wave, lane);
    __syncthreads();
    dense_tanh(act[1], act[0], w3, sb3, 32 * wave, lane);
    __syncthreads();
    dense_tanh(act[0], act[1], w4, sb4, 16 * wave, lane);
    __syncthreads();
    {
      // layer 5 (FP32, linear), split over the wavefronts: wavefront w sums
      // inputs 16 w .. 16 w + 15 of the lane's cell (two 16-byte LDS reads)
      typedef _Float16 half8 __attribute__((ext_vector_type(8)));
      const half8* src = reinterpret_cast<const half8*>(&act[1][lane][16 * wave]);
      const half8 h0 = src[0], h1 = src[1];
      float q[kOut] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const float h = static_cast<float>(j < 8 ? h0[j] : h1[j - 8]);
#pragma unroll
        for (int k = 0; k < kOut; ++k) q[k] = fmaf(sw5[k][16 * wave + j], h, q[k]);
      }
#pragma unroll
      for (int k = 0; k < kOut; ++k) part[wave][k][lane] = q[k];
    }
    __syncthreads();
    if (wave == 0) {
      // the lane's cell: bias plus the four partial sums in wavefront order
      float o[kOut];
#pragma unroll
      for (int k = 0; k < kOut; ++k)
        o[k] = sb5[k] + ((part[0][k][lane] + part[1][k][lane]) + (part[2][k][lane] + part[3][k][lane]));
      if constexpr (!CORRECT) {
        if (live) {
          const size_t c = (size_t)y * nx + x;
#pragma unroll
          for (int k = 0; k < kOut; ++k)
            if (a.out[k]) a.out[k][c] = o[k];
        }
      } else if (m) {
        T* pop = reinterpret_cast<T*>(a.pop);
        float f[9];
        pull_cell<S>(pop, (size_t)nx * ny, nx, ny, x, y, a.rho0, f);
        const float rho = density(f);
        float jx, jy;
        momentum(f, jx, jy);
        const float ux = jx / rho, uy = jy / rho;
        const float r2 = fmaf(a.beta, o[0] - rho, rho);
        const float ux2 = fmaf(a.beta, o[1] - ux, ux);
        const float uy2 = fmaf(a.beta, o[2] - uy, uy);
        float e0[9], e1[9];
        equilibrium32(rho, ux, uy, e0);
        equilibrium32(r2, ux2, uy2, e1);
#pragma unroll
        for (int i = 0; i < 9; ++i)
          store_pulled<S>(pop, nx, ny, x, y, i, f[i] + (e1[i] - e0[i]), a.rho0);
      }
    }
    __syncthreads();  // the next tile reuses the activations
  }
}

// FP64 density of every cell (summed in index order, as the diagnostics do).
template <class S>
__global__ __launch_bounds__(256) void k_rho64(const typename S::T* __restrict__ src, int nx,
                                               int ny, float rho0, double* __restrict__ rho) {
  const size_t n = (size_t)nx * ny;
  for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    float f[9];
    pull_cell<S>(src, n, nx, ny, (int)(c % nx), (int)(c / nx), rho0, f);
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) r += (double)f[i];
    rho[c] = r;
  }
}

// One workgroup per resident slot (the kernel loops over tiles), so that
// every workgroup starts at once and the tiles divide evenly among them.
int pinn_grid(const void* fn, int nx, int ny) {
  const long tiles = (long)((nx + kTile - 1) / kTile) * ny;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return (int)std::max<long>(1, std::min<long>(tiles, (long)per_cu * device_cu_count()));
}

template <bool CORRECT, class F>
hipError_t with_pinn_storage(int storage, F&& f) {
  switch (storage) {
    case LBM_F32: return f(StoreF32{});
    case LBM_F16_SHIFTED: return f(StoreF16S{});
    case LBM_F16_CELL: return f(StoreF16C{});
    default: return hipErrorInvalidValue;  // moment records are not written one value at a time
  }
}

}  // namespace
}  // namespace sclbm

using namespace sclbm;

extern "C" {

lbm_status lbm_pinn_infer(lbm_ctx* c, const float* params, float* rho, float* ux, float* uy) {
  return guarded("lbm_pinn_infer", [&]() -> lbm_status {
    if (!c || !params) return fail(LBM_EINVAL, "ctx or params is NULL");
    if ((uintptr_t)params & 3) return fail(LBM_EINVAL, "params must be 4-byte aligned");
    if (!rho && !ux && !uy) return LBM_OK;
    PinnArgs a{};
    a.params = params;
    a.out[0] = rho;
    a.out[1] = ux;
    a.out[2] = uy;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    const void* fn = reinterpret_cast<const void*>(&k_pinn<StoreF32, false>);
    hipLaunchKernelGGL((k_pinn<StoreF32, false>), dim3(pinn_grid(fn, a.nx, a.ny)), dim3(kThreads),
                       0, c->stream, a);
    SCLBM_HIP(hipGetLastError());
    return LBM_OK;
  });
}

lbm_status lbm_pinn_correct(lbm_ctx* c, const float* params, double beta, uint8_t* mask) {
  return guarded("lbm_pinn_correct", [&]() -> lbm_status {
    if (!c || !params) return fail(LBM_EINVAL, "ctx or params is NULL");
    if ((uintptr_t)params & 3) return fail(LBM_EINVAL, "params must be 4-byte aligned");
    if (!(beta >= 0.0 && beta <= 1.0)) return fail(LBM_EINVAL, "beta must be in [0, 1]");
    if (c->batch) return fail(LBM_EBUSY, "context is a member of a live batch");
    if (c->p.storage == LBM_F16_MOMENT)
      return fail(LBM_EINVAL,
                  "the correction rewrites single stored values; moment storage keeps whole records");
    PinnArgs a{};
    a.pop = c->pop[c->parity];
    a.params = params;
    a.mask = mask;
    a.nx = c->p.nx;
    a.ny = c->p.ny;
    a.rho0 = c->host_desc().rho0;
    a.beta = (float)beta;
    // FP64 density of the state in the idle buffer, then the fused network and
    // correction
    double* rho64 = reinterpret_cast<double*>(c->pop[c->parity ^ 1]);
    a.rho64 = rho64;
    const size_t n = (size_t)a.nx * a.ny;
    const int g = (int)std::min<size_t>((n + 255) / 256, 8192);
    const hipError_t e = with_pinn_storage<true>(c->p.storage, [&](auto tag) {
      using S = decltype(tag);
      hipLaunchKernelGGL(k_rho64<S>, dim3(g), dim3(256), 0, c->stream,
                         reinterpret_cast<const typename S::T*>(a.pop), a.nx, a.ny, a.rho0, rho64);
      const void* fn = reinterpret_cast<const void*>(&k_pinn<S, true>);
      hipLaunchKernelGGL((k_pinn<S, true>), dim3(pinn_grid(fn, a.nx, a.ny)), dim3(kThreads), 0,
                         c->stream, a);
      return hipGetLastError();
    });
    SCLBM_HIP(e);
    return LBM_OK;
  });
}

}  // extern "C"

// sc_device.h -- device-side types and the per-cell arithmetic of the D2Q9
// Shan-Chen step (Li & Zhang, arXiv 2504.10539, Sec. II-A, Eq. (1)).
//
// One inlined cell update is shared by the single-run and the batched step
// kernels, so a simulation's result does not depend on which launch path or
// tile shape advanced it.  The library is compiled with -ffp-contract=off;
// every fused multiply-add below is written out, which keeps the arithmetic
// identical in every kernel that inlines it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sclbm {

// D2Q9 weights in FP32 (4/9, 1/9, 1/36).
constexpr float kW0 = 4.0f / 9.0f;
constexpr float kW1 = 1.0f / 9.0f;
constexpr float kW2 = 1.0f / 36.0f;

// Per-simulation record read by the step kernels.  pop[0]/pop[1] are the two
// population buffers; the state before launch `sub` of a sequence sits in
// pop[(parity + sub) & 1].  nsub is the number of time steps of the sequence
// (the steps of one batched tick): single-step launches run while sub <
// nsub; two-step launches while sub < nsub / 2; with two-step launches an odd
// nsub ends with one single-step tail launch (sub = kTailSub).
struct InstDesc {
  uint64_t pop[2];
  int32_t nx, ny;
  float G, tau, omega, rho0;
  int32_t parity;
  int32_t nsub;
  int64_t remaining;  // batched runs: steps still to take
  int64_t steps;      // batched runs: steps taken
  int32_t storage;
  int32_t per_launch;  // batched runs: steps per launch of the batch's step kernel (1, 2, 3)
  // Address of a 32-bit status word that a step kernel sets to 1 when it
  // meets a cell whose density is not finite or not positive (0: no word).
  // The serving loop points it at pinned host memory and retires such a run
  // early instead of stepping it to the end.
  uint64_t flag;
};
static_assert(sizeof(InstDesc) == 80, "InstDesc layout");

constexpr int kTailSub = -1;   // the single step after a tick's multi-step launches
constexpr int kTail2Sub = -2;  // the two steps after a tick's three-step launches

// Steps per launch of the batch step kernel this simulation runs under (1
// outside batches).
__host__ __device__ __forceinline__ int launch_steps(const InstDesc* d) {
  return d->per_launch > 1 ? d->per_launch : 1;
}
// Whether single-step launch `sub` runs for this simulation, and the buffer
// it reads: the sub-th launch of a single-step tick, or (kTailSub) the last
// step of a tick of nsub / K multi-step launches when nsub mod K is 1.
__host__ __device__ __forceinline__ bool step_runs(const InstDesc* d, int sub) {
  return sub >= 0 ? sub < d->nsub : d->nsub % launch_steps(d) == 1;
}
__host__ __device__ __forceinline__ int step_parity(const InstDesc* d, int sub) {
  return (d->parity + (sub >= 0 ? sub : d->nsub / launch_steps(d))) & 1;
}
// Whether two-step launch `sub` runs: the sub-th launch of a two-step tick,
// or (kTail2Sub) the last two steps of a tick of three-step launches.
__host__ __device__ __forceinline__ bool pair_runs(const InstDesc* d, int sub) {
  return sub >= 0 ? sub < (d->nsub >> 1) : d->nsub % 3 == 2;
}
// The buffer a two- or three-step launch reads: pop[(parity + sub) & 1], or
// for the two-step tail the one the nsub / 3 three-step launches left.
__host__ __device__ __forceinline__ int pair_parity(const InstDesc* d, int sub) {
  return (d->parity + (sub >= 0 ? sub : d->nsub / 3)) & 1;
}
// Whether launch `sub` of a tick of k-step launches (k >= 3) runs.
__host__ __device__ __forceinline__ bool multi_runs(const InstDesc* d, int sub, int k) {
  return sub < d->nsub / k;
}
// Buffer swaps of a tick of n steps with K-step launches: one per launch,
// the steps left over in one further launch.
__host__ __device__ __forceinline__ int64_t tick_flips(int64_t n, int k) {
  return k == 3 ? n / 3 + (n % 3 != 0) : (k == 2 ? (n >> 1) + (n & 1) : n);
}

// One unit of step-kernel work: rows [y0, y0 + h) of the strip of columns
// starting at x0 of simulation `inst`, marched downwards (dir = 0, from y0)
// or upwards (dir = 1, from y0 + h - 1).
struct TileItem {
  int32_t inst, x0, y0;
  int16_t h, dir;
};
static_assert(sizeof(TileItem) == 16, "TileItem layout");

// ------------------------------------------------------------------ layout
//
// Populations live in one buffer of 9 * nx * ny elements.  Row-interleaved
// layout (SCLBM_ROW_LAYOUT = 1, the default): row y of population i starts
// at element (9 y + i) nx, so the nine rows a step touches around one lattice
// row are neighbours in memory; plane-major layout (0): plane i of nx * ny
// elements, row y at (i ny + y) nx.  Either way x is fastest, so a wavefront
// reads and writes consecutive addresses.  Callers see the plane-major
// order only (lbm_get_state / lbm_set_state convert).
#ifndef SCLBM_ROW_LAYOUT
#define SCLBM_ROW_LAYOUT 1
#endif

__host__ __device__ __forceinline__ uint64_t row_index(int i, int y, int nx, int ny) {
#if SCLBM_ROW_LAYOUT
  (void)ny;
  return ((uint64_t)y * 9u + (uint64_t)i) * (uint64_t)nx;
#else
  return ((uint64_t)i * (uint64_t)ny + (uint64_t)y) * (uint64_t)nx;
#endif
}

__host__ __device__ __forceinline__ uint64_t pop_index(int i, int x, int y, int nx, int ny) {
  return row_index(i, y, nx, ny) + (uint64_t)x;
}

// Per-cell-shift storage keeps one more plane after the nine populations:
// rhohat(x), the reference density of the cell that wrote the nine values
// stored at x.  Row y of that plane starts at element 9 nx ny + y nx.
__host__ __device__ __forceinline__ uint64_t rhat_row(int y, int nx, int ny) {
  return 9ull * (uint64_t)nx * (uint64_t)ny + (uint64_t)y * (uint64_t)nx;
}

// ------------------------------------------------------------------ storage

// half(v - w r) rounded once from the exact value (ties to even): one
// mixed-precision FMA with a half-precision result (v_fma_mixlo_f16), w
// uniform across the wavefront.  Written out rather than left to the
// compiler, which fuses a half conversion of an FMA into this instruction
// only where both sit in one basic block: elsewhere the difference is
// rounded twice, and two kernels could then store different halves for the
// same value.
__device__ __forceinline__ _Float16 half_of_fma(float v, float w, float r) {
  uint32_t o;
  asm("v_fma_mixlo_f16 %0, -%1, %2, %3" : "=v"(o) : "s"(w), "v"(r), "v"(v));
  return __builtin_bit_cast(_Float16, (uint16_t)o);
}

// FP32 populations.  Stores stream past the caches (the buffer written is
// read again only by the next step).
struct StoreF32 {
  using T = float;
  static constexpr int kBytes = 4;
  static constexpr bool kStream = true;
  static constexpr bool kCellShift = false;
  static constexpr bool kMoment = false;
  template <class P>
  __device__ static __forceinline__ float load(P p, float /*shift*/) { return *p; }
  __device__ static __forceinline__ T pack(float v, float /*shift*/) { return v; }
};

// FP16 populations holding f_i - w_i rho0, widened back to FP32 on load.
struct StoreF16S {
  using T = _Float16;
  static constexpr int kBytes = 2;
  static constexpr bool kStream = false;
  static constexpr bool kCellShift = false;
  static constexpr bool kMoment = false;
  template <class P>
  __device__ static __forceinline__ float load(P p, float shift) {
    return static_cast<float>(*p) + shift;
  }
  __device__ static __forceinline__ T pack(float v, float shift) {
    return static_cast<T>(v - shift);  // v_cvt_f16_f32: round to nearest even
  }
};

// FP16 populations shifted per cell: the nine values a cell stores hold
// half(f_i - w_i rhohat) (rounded once), where rhohat = half(rho) of that
// (writing) cell and is
// stored beside them (rhat_row).  Read back as rhohat * w_i + h, rounded
// once.  Only the non-equilibrium and velocity parts of f_i are left to round
// to half precision, in either phase.
struct StoreF16C {
  using T = _Float16;
  static constexpr int kBytes = 2;
  static constexpr bool kStream = false;
  static constexpr bool kCellShift = true;
  static constexpr bool kMoment = false;
  __device__ static __forceinline__ float decode(T h, T rh, float w) {
    return __builtin_fmaf(static_cast<float>(rh), w, static_cast<float>(h));
  }
  // half(v - w rhohat): the compiler fuses the conversion into the FMA
  // (v_fma_mixlo_f16, one rounding) in every kernel that stores this form;
  // written as half_of_fma it costs the four-wave two-step kernel a spilled
  // register.  The tile-shape tests check that every kernel stores the same
  // halves.
  __device__ static __forceinline__ T encode(float v, T rh, float w) {
    return static_cast<T>(__builtin_fmaf(-w, static_cast<float>(rh), v));
  }
  __device__ static __forceinline__ T ref(float rho) { return static_cast<T>(rho); }
};

// FP16 populations with exact conserved moments.  A cell x keeps a record of
// the nine values A_i(x) it wrote: its density rho (the mass of the record)
// and the momentum jx, jy of the A_i in FP32, and A_3 .. A_8 as
// h_i = half(A_i - w_i rho) (rounded once, half_of_fma).  A_1 and A_2 are rebuilt
// from the momentum and A_0 from the mass (mom_decode), so the mass and
// momentum a cell hands on to its neighbours are exact up to FP32 rounding and
// only non-conserved moments round to half precision; the BGK collision
// relaxes those towards equilibrium instead of carrying the rounding on.
// 24 bytes per cell (layout: mom_row).
struct StoreF16M {
  using T = _Float16;  // the six FP16 rows
  static constexpr int kBytes = 2;
  static constexpr bool kStream = false;
  static constexpr bool kCellShift = false;
  static constexpr bool kMoment = true;
};

// Moment-storage layout: lattice row y occupies 24 nx bytes from byte
// 24 nx y: the FP32 rows of rho, jx and jy (mom_f32, k = 0, 1, 2), then the
// FP16 rows of h_3 .. h_8 (mom_f16, i = 3 .. 8); x is fastest in every row.
__host__ __device__ __forceinline__ uint64_t mom_row(int y, int nx) {
  return 24ull * (uint64_t)nx * (uint64_t)y;
}
__host__ __device__ __forceinline__ uint64_t mom_f32(int k, int nx) {
  return 4ull * (uint64_t)nx * (uint64_t)k;
}
__host__ __device__ __forceinline__ uint64_t mom_f16(int i, int nx) {
  return 12ull * (uint64_t)nx + 2ull * (uint64_t)nx * (uint64_t)(i - 3);
}

// Pointer into global memory (address space 1): loads and stores through it
// use the global_* instructions with a scalar base and a 32-bit lane offset.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> as_global(uint64_t a) {
  return reinterpret_cast<gptr<T>>(a);
}

__device__ __forceinline__ int wrap_dec(int a, int n) { return a == 0 ? n - 1 : a - 1; }
__device__ __forceinline__ int wrap_inc(int a, int n) { return a == n - 1 ? 0 : a + 1; }

// ------------------------------------------------------------------ arithmetic

// Density: the populations summed in index order.
__device__ __forceinline__ float density(const float f[9]) {
  float r = f[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) r += f[i];
  return r;
}

// Pseudopotential psi(rho) = 1 - exp(-rho).  exp(-rho) = 2^(p + d) with
// p = fl(-rho L), L = log2(e) rounded to FP32, and d the rest of -rho log2(e):
// the exact residual of that product (one FMA) plus -rho times the part of
// log2(e) beyond L.  2^p comes from the hardware base-2 exponential
// (v_exp_f32) and d enters to first order, 2^(p + d) = 2^p (1 + d ln 2) up to
// a relative (d ln 2)^2 / 2 < 1e-14.  Seven instructions where the library
// exp takes thirteen (its range reduction guards arguments far outside what a
// density reaches).
__device__ __forceinline__ float psi_of(float rho) {
  constexpr float kLog2e = 1.44269502f;      // fl(log2 e)
  constexpr float kLog2eLo = 1.92596299e-8f;  // log2 e - fl(log2 e)
  constexpr float kLn2 = 0.693147182f;
  const float p = -rho * kLog2e;
  const float d = fmaf(-rho, kLog2eLo, fmaf(-rho, kLog2e, -p));
  const float e = __builtin_amdgcn_exp2f(p);
  return 1.0f - fmaf(e, d * kLn2, e);
}

// 1.0f that the compiler cannot see through: h * one + s then keeps its FMA
// form, with h widened from half precision, and is selected as one
// mixed-precision FMA (v_fma_mix_f32) instead of a conversion and an add.
// The product is exact, so the result equals float(h) + s.
__device__ __forceinline__ float opaque_one() {
  float r = 1.0f;
  asm("" : "+s"(r));
  return r;
}

// Interaction force F = -G psi(x) sum_i w_i psi(x + e_i) e_i.  The stencil
// sum is taken as differences of opposite neighbours first: neighbouring psi
// values are close, so each difference is exact in FP32 and the sum keeps
// the antisymmetry of the pair force instead of cancelling large partial
// sums.
__device__ __forceinline__ void force_of(float pc, float pE, float pN, float pW, float pS,
                                         float pNE, float pNW, float pSW, float pSE, float G,
                                         float& Fx, float& Fy) {
  const float dA = pNE - pSW;  // e5 against e7
  const float dB = pSE - pNW;  // e8 against e6
  const float sx = fmaf(kW1, pE - pW, kW2 * (dA + dB));
  const float sy = fmaf(kW1, pN - pS, kW2 * (dA - dB));
  const float gp = -G * pc;
  Fx = gp * sx;
  Fy = gp * sy;
}

// Momentum j = sum_i f_i e_i, as differences of opposite populations.
__device__ __forceinline__ void momentum(const float f[9], float& jx, float& jy) {
  const float a = f[5] - f[7];
  const float b = f[8] - f[6];
  jx = (f[1] - f[3]) + (a + b);
  jy = (f[2] - f[4]) + (a - b);
}

// Moment storage (StoreF16M): A_i = rho w_i + h_i for i = 3 .. 8, rounded once.
__device__ __forceinline__ float mom_pop(float rho, _Float16 h, float w) {
  return __builtin_fmaf(rho, w, static_cast<float>(h));
}
// A_1 of a record from its rho, jx and h_3, h_5 .. h_8: jx = A_1 - A_3 +
// (A_5 - A_7) + (A_8 - A_6), solved for A_1 in that grouping.
__device__ __forceinline__ float mom_a1(float rho, float jx, _Float16 h3, _Float16 h5, _Float16 h6,
                                        _Float16 h7, _Float16 h8) {
  const float a3 = mom_pop(rho, h3, kW1);
  const float d = mom_pop(rho, h5, kW2) - mom_pop(rho, h7, kW2);
  const float e = mom_pop(rho, h8, kW2) - mom_pop(rho, h6, kW2);
  return (jx + a3) - (d + e);
}
// A_2 from rho, jy and h_4 .. h_8: jy = A_2 - A_4 + (A_5 - A_7) - (A_8 - A_6).
__device__ __forceinline__ float mom_a2(float rho, float jy, _Float16 h4, _Float16 h5, _Float16 h6,
                                        _Float16 h7, _Float16 h8) {
  const float a4 = mom_pop(rho, h4, kW1);
  const float d = mom_pop(rho, h5, kW2) - mom_pop(rho, h7, kW2);
  const float e = mom_pop(rho, h8, kW2) - mom_pop(rho, h6, kW2);
  return (jy + a4) - (d - e);
}
// A_0 from the record's mass: rho minus the other eight values, summed in the
// grouping of the collision's mass balance.
__device__ __forceinline__ float mom_a0(float rho, const float (&a)[9]) {
  return rho - (((a[1] + a[3]) + (a[2] + a[4])) + ((a[5] + a[7]) + (a[6] + a[8])));
}
// All nine values of a record (bitwise the values mom_a1, mom_a2 and mom_pop
// give one at a time).
__device__ __forceinline__ void mom_decode(float rho, float jx, float jy, const _Float16 (&h)[6],
                                           float (&a)[9]) {
  a[3] = mom_pop(rho, h[0], kW1);
  a[4] = mom_pop(rho, h[1], kW1);
  a[5] = mom_pop(rho, h[2], kW2);
  a[6] = mom_pop(rho, h[3], kW2);
  a[7] = mom_pop(rho, h[4], kW2);
  a[8] = mom_pop(rho, h[5], kW2);
  const float d = a[5] - a[7], e = a[8] - a[6];
  a[1] = (jx + a[3]) - (d + e);
  a[2] = (jy + a[4]) - (d - e);
  a[0] = mom_a0(rho, a);
}
// The record of the values v written by a cell whose mass is rho (the
// density it collided with, which the BGK collision conserves).
__device__ __forceinline__ void mom_encode(const float* v, float rho, float& jx, float& jy,
                                           _Float16 (&h)[6]) {
  momentum(v, jx, jy);
  h[0] = half_of_fma(v[3], kW1, rho);
  h[1] = half_of_fma(v[4], kW1, rho);
  h[2] = half_of_fma(v[5], kW2, rho);
  h[3] = half_of_fma(v[6], kW2, rho);
  h[4] = half_of_fma(v[7], kW2, rho);
  h[5] = half_of_fma(v[8], kW2, rho);
}

// 1 / x from the hardware reciprocal (within 1 ulp) and one FMA correction
// with its exact residual: the correctly rounded quotient (Markstein's
// correction of a faithful reciprocal).  Compared against the IEEE division
// on gfx950 for every positive normal float: bitwise equal for all x < 2^126,
// so for any density a finite run can reach; above that, where 1 / x is
// subnormal, the two may differ.  Three instructions instead of the division
// sequence: 5% fewer VALU instructions in the FP16-shifted two-step kernel,
// which instruction issue bounds.
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}

// Divergence check of a collided cell: the lanes (of this wavefront) whose
// density is NaN, infinite, zero or negative, among the lanes where `live`
// holds.  One class test per cell (mask: signalling and quiet NaN, -inf,
// negative normal and subnormal, -0, +0, +inf).
constexpr int kUnstableClass = 0x27F;
__device__ __forceinline__ uint64_t unstable_lanes(float rho, bool live) {
  return __builtin_amdgcn_ballot_w64(live && __builtin_amdgcn_classf(rho, kUnstableClass));
}
// Sets the run's status word if this wavefront met an unstable cell.  Called
// once per work item with every lane active; the store is a plain vector store
// of the same value from each such wavefront.
__device__ __forceinline__ void report_unstable(const InstDesc* dp, uint64_t bad) {
  if (bad != 0 && (threadIdx.x & 63) == 0) {
    const uint64_t a = dp->flag;
    if (a != 0) *reinterpret_cast<volatile int*>(a) = 1;
  }
}

// BGK collision with the Shan-Chen velocity shift, in place on f:
//   u_eq = (j + tau F) / rho,
//   f_eq_i = w_i rho (1 + 3 e_i.u + 4.5 (e_i.u)^2 - 1.5 u.u)  (i = 1..8),
//   f_eq_0 = rho - sum_{i>0} f_eq_i   (mass balance: the rounded weights do
//                                      not sum to one in FP32),
//   f*_i = f_i + (f_eq_i - f_i) / tau.
__device__ __forceinline__ void collide(float f[9], float rho, float Fx, float Fy, float tau,
                                        float omega) {
  float jx, jy;
  momentum(f, jx, jy);
  const float inv = recip(rho);
  const float ux = fmaf(tau, Fx, jx) * inv;
  const float uy = fmaf(tau, Fy, jy) * inv;
  const float base = fmaf(-1.5f, fmaf(ux, ux, uy * uy), 1.0f);
  // w_1 rho and w_5 rho as the correctly rounded quotients rho / 9 and
  // rho / 36: the estimate kW1 * rho plus one FMA correction with its exact
  // residual.  The FP32 weights themselves are 7.45e-9 too large, and that
  // one-signed bias in every moving equilibrium population measurably drifts
  // the interfaces over thousands of steps.  rho / 36 = (rho / 9) / 4 exactly.
  const float q9 = kW1 * rho;
  const float r1 = fmaf(fmaf(-q9, 9.0f, rho), kW1, q9);
  const float r2 = 0.25f * r1;
  float feq[9];
  {
    const float s = fmaf(4.5f * ux, ux, base), t = 3.0f * ux;
    feq[1] = r1 * (s + t);
    feq[3] = r1 * (s - t);
  }
  {
    const float s = fmaf(4.5f * uy, uy, base), t = 3.0f * uy;
    feq[2] = r1 * (s + t);
    feq[4] = r1 * (s - t);
  }
  {
    const float v = ux + uy;
    const float s = fmaf(4.5f * v, v, base), t = 3.0f * v;
    feq[5] = r2 * (s + t);
    feq[7] = r2 * (s - t);
  }
  {
    const float v = uy - ux;  // e6 = (-1, 1); e8 = -e6
    const float s = fmaf(4.5f * v, v, base), t = 3.0f * v;
    feq[6] = r2 * (s + t);
    feq[8] = r2 * (s - t);
  }
  feq[0] = rho - (((feq[1] + feq[3]) + (feq[2] + feq[4])) + ((feq[5] + feq[7]) + (feq[6] + feq[8])));
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = fmaf(omega, feq[i] - f[i], f[i]);
}


// ------------------------------------------------------------------ one cell at a time

// Pre-collision populations at cell (x, y), pulled from a buffer.
template <class S>
__device__ __forceinline__ void pull_cell(const typename S::T* src, size_t n, int nx, int ny, int x,
                                          int y, float rho0, float f[9]) {
  (void)n;
  const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
  const int ym = wrap_dec(y, ny), yp = wrap_inc(y, ny);
  if constexpr (S::kMoment) {
    const char* b = reinterpret_cast<const char*>(src);
    auto F = [&](int k, int xx, int yy) {
      return *reinterpret_cast<const float*>(b + mom_row(yy, nx) + mom_f32(k, nx) + 4ull * xx);
    };
    auto H = [&](int i, int xx, int yy) {
      return *reinterpret_cast<const _Float16*>(b + mom_row(yy, nx) + mom_f16(i, nx) + 2ull * xx);
    };
    _Float16 h[6];
#pragma unroll
    for (int i = 3; i < 9; ++i) h[i - 3] = H(i, x, y);
    float own[9];
    mom_decode(F(0, x, y), F(1, x, y), F(2, x, y), h, own);
    f[0] = own[0];
    f[1] = mom_a1(F(0, xm, y), F(1, xm, y), H(3, xm, y), H(5, xm, y), H(6, xm, y), H(7, xm, y),
                  H(8, xm, y));
    f[2] = mom_a2(F(0, x, ym), F(2, x, ym), H(4, x, ym), H(5, x, ym), H(6, x, ym), H(7, x, ym),
                  H(8, x, ym));
    f[3] = mom_pop(F(0, xp, y), H(3, xp, y), kW1);
    f[4] = mom_pop(F(0, x, yp), H(4, x, yp), kW1);
    f[5] = mom_pop(F(0, xm, ym), H(5, xm, ym), kW2);
    f[6] = mom_pop(F(0, xp, ym), H(6, xp, ym), kW2);
    f[7] = mom_pop(F(0, xp, yp), H(7, xp, yp), kW2);
    f[8] = mom_pop(F(0, xm, yp), H(8, xm, yp), kW2);
  } else {
    const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
    const int sx[9] = {x, xm, x, xp, x, xm, xp, xp, xm};
    const int sy[9] = {y, y, ym, y, yp, ym, ym, yp, yp};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if constexpr (S::kCellShift)
        f[i] = S::decode(src[pop_index(i, sx[i], sy[i], nx, ny)],
                         src[rhat_row(sy[i], nx, ny) + (uint64_t)sx[i]], ws[i]);
      else
        f[i] = S::load(src + pop_index(i, sx[i], sy[i], nx, ny), ws[i] * rho0);
    }
  }
}


// Writes v as the stored value a pull of population i at cell (x, y) reads,
// A_i(x - e_i), rounded as the storage form rounds it (per-cell-shift
// storage: with the reference density of the cell that holds it, which is
// kept).  Moment storage keeps whole records and has no single stored value
// per population; it is not written this way.
template <class S>
__device__ __forceinline__ void store_pulled(typename S::T* dst, int nx, int ny, int x, int y,
                                             int i, float v, float rho0) {
  static_assert(!S::kMoment, "moment records are written whole");
  const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
  int sx = x - ex[i], sy = y - ey[i];
  sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
  sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
  const uint64_t at = pop_index(i, sx, sy, nx, ny);
  if constexpr (S::kCellShift)
    dst[at] = S::encode(v, dst[rhat_row(sy, nx, ny) + (uint64_t)sx], ws[i]);
  else
    dst[at] = S::pack(v, ws[i] * rho0);
}

}  // namespace sclbm

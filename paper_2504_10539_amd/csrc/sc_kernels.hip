// sc_kernels.hip -- gfx950 kernels of the D2Q9 Shan-Chen step and its
// diagnostics (Li & Zhang, arXiv 2504.10539: Sec. II-A Eq. (1); Sec. III-A
// initial droplet; Sec. II-D Eqs. (9)-(13) and Sec. IV-E Eqs. (14)-(16)).
//
// Population buffers hold the nine populations structure-of-arrays, in the
// layout of row_index() (sc_device.h).  A buffer holds post-collision values
// at the cell they leave from, so the pre-collision state is read by pulling:
// f_i(x, t) = A_i(x - e_i).  One step reads A and writes the other buffer B
// at the cell itself; the next step swaps the roles.

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "sc_device.h"
#include "sc_launch.h"

namespace sclbm {

// ============================================================== FP64 diagnostics per cell

// FP64 density: the widened populations summed in index order.
__device__ __forceinline__ double density64(const float (&f)[10]) {
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) r += (double)f[i];
  return r;
}

// Accumulators of the diagnostics: mass, mom_x, mom_y, bad cells, cells above
// the threshold, max |grad rho|, sum |grad rho|, sum |grad rho|^2, rho max, min.
__device__ __forceinline__ void diag_zero(double (&acc)[10]) {
#pragma unroll
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  acc[8] = -INFINITY;
  acc[9] = INFINITY;
}

// Diagnostics of one cell (its pre-collision populations f; FP64 rho of the
// rows below, at and above it in dn, md, up, column c): Eq. (16) with
// periodic wrap, threshold of Eq. (9) strict.
__device__ __forceinline__ void diag_cell(double (&acc)[10], const float (&f)[10], int c, int cl,
                                          int cr, const double* dn, const double* md,
                                          const double* up) {
  bool fin = true;
#pragma unroll
  for (int i = 0; i < 9; ++i) fin = fin && isfinite(f[i]);
  const double r = md[c];
  const double jx = ((double)f[1] - (double)f[3]) + ((double)f[5] - (double)f[6]) +
                    ((double)f[8] - (double)f[7]);
  const double jy = ((double)f[2] - (double)f[4]) + ((double)f[5] - (double)f[8]) +
                    ((double)f[6] - (double)f[7]);
  const double gx = (md[cr] - md[cl]) / 2.0;
  const double gy = (up[c] - dn[c]) / 2.0;
  const double g = sqrt(gx * gx + gy * gy);
  acc[0] += r;
  acc[1] += jx;
  acc[2] += jy;
  if (!fin || !(r > 0.0)) acc[3] += 1.0;
  if (g > 0.01) acc[4] += 1.0;
  acc[5] = fmax(acc[5], g);
  acc[6] += g;
  acc[7] += g * g;
  acc[8] = fmax(acc[8], r);
  acc[9] = fmin(acc[9], r);
}

// ============================================================== step kernel
//
// A workgroup of NT threads owns a strip of SW = NT * CPT columns (thread t
// holds columns x0 + t + k NT, k < CPT, so every load and store instruction
// of a wavefront covers consecutive addresses) and marches down `h` rows.
// Per row it pulls the nine populations of the next row, forms rho and psi,
// and puts psi in a four-row LDS ring; after one barrier it has psi on the
// 3x3 neighbourhood of the current row and collides it.  Each population of
// the strip is read from HBM once; the extra reads are one halo column on
// each side (two lanes) and one halo row above and below the band.  PF rows
// of loads are kept in flight ahead of the row being finished.

// DIAG = true: the launch also accumulates, from the same pulled populations,
// the FP64 interface diagnostics of the state it advances (the quantities of
// the separate diagnostics pass, per cell in the same arithmetic); rho in FP64
// goes through a second LDS ring for the Eq. (16) gradient.
template <class S, int NT, int CPT, bool DIAG = false>
struct Strip {
  using T = typename S::T;
  static constexpr int SW = NT * CPT;
  static constexpr int kCPT = CPT;
  static constexpr bool kDiag = DIAG;
  using RhoRing = double (*)[SW + 2];

  uint64_t src, dst;  // buffer base addresses (read / written this step)
  float sh[9];
  int nx, ny, x0, y0, h, dir, wcols;
  // Columns of this lane's cells; slot CPT is the halo column (lanes 0, 1).
  int xc[CPT + 1], xm[CPT + 1], xp[CPT + 1];
  bool live[CPT + 1];
  float G, tau, omega;
  uint64_t bad;  // lanes that collided a cell with a non-finite or non-positive density
  // DIAG accumulators: mass, mom_x, mom_y, bad cells, cells above the
  // threshold, max |grad rho|, sum |grad rho|, sum |grad rho|^2, rho max, min.
  double acc[10];

  // First element of row y of population i.  The address is the same for the
  // whole workgroup; readfirstlane keeps it in scalar registers, so each load
  // and store is a scalar base plus the lane's 32-bit column offset.
  __device__ __forceinline__ static uint64_t uniform(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
  }
  __device__ __forceinline__ gptr<const T> in_row(int i, int y) const {
    return as_global<const T>(uniform(src + row_index(i, y, nx, ny) * sizeof(T)));
  }
  __device__ __forceinline__ gptr<T> out_row(int i, int y) const {
    return as_global<T>(uniform(dst + row_index(i, y, nx, ny) * sizeof(T)));
  }
  // Row y of the reference-density plane (per-cell-shift storage).
  __device__ __forceinline__ gptr<const T> rhat_in(int y) const {
    return as_global<const T>(uniform(src + rhat_row(y, nx, ny) * sizeof(T)));
  }
  __device__ __forceinline__ gptr<T> rhat_out(int y) const {
    return as_global<T>(uniform(dst + rhat_row(y, nx, ny) * sizeof(T)));
  }

  __device__ __forceinline__ void setup(const InstDesc* __restrict__ dp, const TileItem& ti,
                                        int sub) {
    nx = dp->nx;
    ny = dp->ny;
    x0 = ti.x0;
    y0 = ti.y0;
    h = ti.h;
    dir = ti.dir;
    wcols = min(SW, nx - x0);
    bad = 0;
    G = dp->G;
    tau = dp->tau;
    omega = dp->omega;
    const float rho0 = dp->rho0;
    const int par = step_parity(dp, sub);
    const uint64_t a = dp->pop[0], b = dp->pop[1];
    src = par ? b : a;
    dst = par ? a : b;
    const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
#pragma unroll
    for (int i = 0; i < 9; ++i) sh[i] = ws[i] * rho0;
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int c = t + k * NT;
      live[k] = c < wcols;
      const int x = live[k] ? x0 + c : x0;
      xc[k] = x;
      xm[k] = wrap_dec(x, nx);
      xp[k] = wrap_inc(x, nx);
    }
    live[CPT] = t < 2;
    {
      const int xl = x0 == 0 ? nx - 1 : x0 - 1;
      const int xr = (x0 + wcols) % nx;
      const int x = t == 0 ? xl : xr;
      xc[CPT] = x;
      xm[CPT] = wrap_dec(x, nx);
      xp[CPT] = wrap_inc(x, nx);
    }
  }

  // A lane's byte offset re-materialised where it is used (an empty asm on a
  // copy), so that each access is formed in the loop body as scalar row base +
  // 32-bit lane offset (global_* with saddr) instead of from a hoisted 64-bit
  // vector offset.
  __device__ __forceinline__ static uint32_t fresh(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
  }

  // Element at byte offset `boff` (32-bit, lane-varying) from a uniform row base.
  __device__ __forceinline__ static gptr<const T> at(gptr<const T> base, uint32_t boff) {
    return reinterpret_cast<gptr<const T>>(reinterpret_cast<gptr<const char>>(base) + boff);
  }
  __device__ __forceinline__ static gptr<T> at(gptr<T> base, uint32_t boff) {
    return reinterpret_cast<gptr<T>>(reinterpret_cast<gptr<char>>(base) + boff);
  }

  // Lattice row of march position j (j = -1 and j = h are the halo rows).
  __device__ __forceinline__ int row_of(int j) const {
    int y = dir ? y0 + h - 1 - j : y0 + j;
    return y < 0 ? y + ny : (y >= ny ? y - ny : y);
  }

  // Moment storage: uniform row addresses of the FP32 row k and the FP16 row of
  // population i of the lattice row that starts at byte address `row`.
  __device__ __forceinline__ gptr<const float> mom_in32(uint64_t row, int k) const {
    return as_global<const float>(uniform(row + mom_f32(k, nx)));
  }
  __device__ __forceinline__ gptr<const T> mom_in16(uint64_t row, int i) const {
    return as_global<const T>(uniform(row + mom_f16(i, nx)));
  }
  template <class U>
  __device__ __forceinline__ static U ldb(gptr<const U> base, uint32_t boff) {
    return *reinterpret_cast<gptr<const U>>(reinterpret_cast<gptr<const char>>(base) + boff);
  }
  template <class U>
  __device__ __forceinline__ static void stb(gptr<U> base, uint32_t boff, U v) {
    *reinterpret_cast<gptr<U>>(reinterpret_cast<gptr<char>>(base) + boff) = v;
  }

  // Moment storage: the pulled populations of row y for every live slot.
  // f_0 is the cell's own record decoded whole; f_1 and f_2 are rebuilt from
  // the momentum of the records at x - e_1 and x - e_2; the others are one
  // value each of the records they come from.
  __device__ __forceinline__ void pull_moments(int y, int ym, int yp,
                                               float (&f)[CPT + 1][10]) const {
    const uint64_t b0 = src + mom_row(y, nx), bm = src + mom_row(ym, nx), bp = src + mom_row(yp, nx);
    const gptr<const float> r0 = mom_in32(b0, 0), jx0 = mom_in32(b0, 1), jy0 = mom_in32(b0, 2),
                            rm = mom_in32(bm, 0), jym = mom_in32(bm, 2), rp = mom_in32(bp, 0);
#pragma unroll
    for (int k = 0; k <= CPT; ++k) {
      if (!live[k]) continue;
      const uint32_t c4 = fresh((uint32_t)xc[k] * 4u), m4 = fresh((uint32_t)xm[k] * 4u),
                     p4 = fresh((uint32_t)xp[k] * 4u);
      const uint32_t c2 = fresh((uint32_t)xc[k] * 2u), m2 = fresh((uint32_t)xm[k] * 2u),
                     p2 = fresh((uint32_t)xp[k] * 2u);
      T h[6];
#pragma unroll
      for (int i = 3; i < 9; ++i) h[i - 3] = ldb(mom_in16(b0, i), c2);
      float own[9];
      mom_decode(ldb(r0, c4), ldb(jx0, c4), ldb(jy0, c4), h, own);
      f[k][0] = own[0];
      f[k][1] = mom_a1(ldb(r0, m4), ldb(jx0, m4), ldb(mom_in16(b0, 3), m2),
                       ldb(mom_in16(b0, 5), m2), ldb(mom_in16(b0, 6), m2),
                       ldb(mom_in16(b0, 7), m2), ldb(mom_in16(b0, 8), m2));
      f[k][2] = mom_a2(ldb(rm, c4), ldb(jym, c4), ldb(mom_in16(bm, 4), c2),
                       ldb(mom_in16(bm, 5), c2), ldb(mom_in16(bm, 6), c2),
                       ldb(mom_in16(bm, 7), c2), ldb(mom_in16(bm, 8), c2));
      f[k][3] = mom_pop(ldb(r0, p4), ldb(mom_in16(b0, 3), p2), kW1);
      f[k][4] = mom_pop(ldb(rp, c4), ldb(mom_in16(bp, 4), c2), kW1);
      f[k][5] = mom_pop(ldb(rm, m4), ldb(mom_in16(bm, 5), m2), kW2);
      f[k][6] = mom_pop(ldb(rm, p4), ldb(mom_in16(bm, 6), p2), kW2);
      f[k][7] = mom_pop(ldb(rp, p4), ldb(mom_in16(bp, 7), p2), kW2);
      f[k][8] = mom_pop(ldb(rp, m4), ldb(mom_in16(bp, 8), m2), kW2);
    }
  }

  // Pre-collision populations of the row at march position j for every live
  // slot: f_i(x, y) = A_i(x - e_i), so population i is read from row y - e_iy.
  __device__ __forceinline__ void pull(int j, float (&f)[CPT + 1][10]) const {
    const int y = row_of(j);
    const int ym = wrap_dec(y, ny), yp = wrap_inc(y, ny);
    if constexpr (S::kMoment) {
      pull_moments(y, ym, yp, f);
    } else {
      const gptr<const T> p0 = in_row(0, y), p1 = in_row(1, y), p2 = in_row(2, ym),
                          p3 = in_row(3, y), p4 = in_row(4, yp), p5 = in_row(5, ym),
                          p6 = in_row(6, ym), p7 = in_row(7, yp), p8 = in_row(8, yp);
      constexpr uint32_t B = sizeof(T);
#pragma unroll
      for (int k = 0; k <= CPT; ++k) {
        if (live[k]) {
          const uint32_t c = fresh((uint32_t)xc[k] * B), m = fresh((uint32_t)xm[k] * B),
                         p = fresh((uint32_t)xp[k] * B);
          if constexpr (S::kCellShift) {
            // each value is decoded with the reference density of the cell it
            // was read from (same row and column in the reference plane)
            const gptr<const T> q0 = rhat_in(y), qm = rhat_in(ym), qp = rhat_in(yp);
            f[k][0] = S::decode(*at(p0, c), *at(q0, c), kW0);
            f[k][1] = S::decode(*at(p1, m), *at(q0, m), kW1);
            f[k][2] = S::decode(*at(p2, c), *at(qm, c), kW1);
            f[k][3] = S::decode(*at(p3, p), *at(q0, p), kW1);
            f[k][4] = S::decode(*at(p4, c), *at(qp, c), kW1);
            f[k][5] = S::decode(*at(p5, m), *at(qm, m), kW2);
            f[k][6] = S::decode(*at(p6, p), *at(qm, p), kW2);
            f[k][7] = S::decode(*at(p7, p), *at(qp, p), kW2);
            f[k][8] = S::decode(*at(p8, m), *at(qp, m), kW2);
          } else {
            f[k][0] = S::load(at(p0, c), sh[0]);
            f[k][1] = S::load(at(p1, m), sh[1]);
            f[k][2] = S::load(at(p2, c), sh[2]);
            f[k][3] = S::load(at(p3, p), sh[3]);
            f[k][4] = S::load(at(p4, c), sh[4]);
            f[k][5] = S::load(at(p5, m), sh[5]);
            f[k][6] = S::load(at(p6, p), sh[6]);
            f[k][7] = S::load(at(p7, p), sh[7]);
            f[k][8] = S::load(at(p8, m), sh[8]);
          }
        }
      }
    }
  }

  // psi of march position j into ring slot (j + 1) & 3 (LDS column index =
  // strip column + 1); the density is kept in slot 9 for the collision.
  __device__ __forceinline__ void publish(int j, float (&f)[CPT + 1][10], float (*ring)[SW + 2],
                                          RhoRing rring = nullptr) const {
    float* row = ring[(j + 1) & 3];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < CPT; ++k)
      if (live[k]) {
        f[k][9] = density(f[k]);
        row[t + k * NT + 1] = psi_of(f[k][9]);
        if constexpr (DIAG) rring[(j + 1) & 3][t + k * NT + 1] = density64(f[k]);
      }
    if (live[CPT]) {
      row[t == 0 ? 0 : wcols + 1] = psi_of(density(f[CPT]));
      if constexpr (DIAG) rring[(j + 1) & 3][t == 0 ? 0 : wcols + 1] = density64(f[CPT]);
    }
  }

  __device__ __forceinline__ static double density64(const float (&f)[10]) {
    return sclbm::density64(f);
  }
  __device__ __forceinline__ void diag_zero() { sclbm::diag_zero(acc); }
  __device__ __forceinline__ void diag_cell(const float (&f)[10], int c, const double* dn,
                                            const double* md, const double* up) {
    sclbm::diag_cell(acc, f, c, c - 1, c + 1, dn, md, up);
  }

  // Collide the row at march position r (psi of positions r-1, r, r+1 already
  // in the ring) and store it.  Marching upwards, the previous position is
  // the row above (y + 1) and the next one the row below.
  __device__ __forceinline__ void finish(int r, float (&f)[CPT + 1][10], const float (*ring)[SW + 2],
                                         RhoRing rring = nullptr) {
    const float* prev = ring[r & 3];
    const float* md = ring[(r + 1) & 3];
    const float* next = ring[(r + 2) & 3];
    const float* dn = dir ? next : prev;
    const float* up = dir ? prev : next;
    if constexpr (DIAG) {
      const double* rp = rring[r & 3];
      const double* rn = rring[(r + 2) & 3];
#pragma unroll
      for (int k = 0; k < CPT; ++k)
        if (live[k])
          diag_cell(f[k], threadIdx.x + k * NT + 1, dir ? rn : rp, rring[(r + 1) & 3], dir ? rp : rn);
    }
    gptr<T> o[9];
    const int y = row_of(r);
#pragma unroll
    for (int i = 0; i < 9; ++i) o[i] = out_row(i, y);
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      if (!live[k]) continue;
      const int c = t + k * NT + 1;
      float Fx, Fy;
      force_of(md[c], md[c + 1], up[c], md[c - 1], dn[c], up[c + 1], up[c - 1], dn[c - 1],
               dn[c + 1], G, Fx, Fy);
      bad |= unstable_lanes(f[k][9], true);
      collide(f[k], f[k][9], Fx, Fy, tau, omega);
      const uint32_t xb = fresh((uint32_t)xc[k] * (uint32_t)sizeof(T));
      if constexpr (S::kMoment) {
        // the record: this cell's density (its mass), the momentum of the
        // collided values and the six FP16 deviations
        float jx, jy;
        T hv[6];
        mom_encode(f[k], f[k][9], jx, jy, hv);
        const uint64_t b = dst + mom_row(y, nx);
        const uint32_t x4 = fresh((uint32_t)xc[k] * 4u);
        stb(as_global<float>(uniform(b + mom_f32(0, nx))), x4, f[k][9]);
        stb(as_global<float>(uniform(b + mom_f32(1, nx))), x4, jx);
        stb(as_global<float>(uniform(b + mom_f32(2, nx))), x4, jy);
#pragma unroll
        for (int i = 3; i < 9; ++i) stb(as_global<T>(uniform(b + mom_f16(i, nx))), xb, hv[i - 3]);
      } else if constexpr (S::kCellShift) {
        const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
        const T rh = S::ref(f[k][9]);  // this cell's reference: half(rho)
#pragma unroll
        for (int i = 0; i < 9; ++i) *at(o[i], xb) = S::encode(f[k][i], rh, ws[i]);
        *at(rhat_out(y), xb) = rh;
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          if constexpr (S::kStream)
            __builtin_nontemporal_store(S::pack(f[k][i], sh[i]), at(o[i], xb));
          else
            *at(o[i], xb) = S::pack(f[k][i], sh[i]);
        }
      }
    }
  }
};

// One band of a strip: PF rows of loads in flight ahead of the row being
// finished; one barrier per row.
template <class St, int PF>
__device__ __forceinline__ void march(St& s, float (*ring)[St::SW + 2],
                                      typename St::RhoRing rring = nullptr) {
  const int h = s.h;
  constexpr int C1 = St::kCPT + 1;  // the lane's cells plus its halo slot
  if constexpr (PF == 1) {
    float a[C1][10], b[C1][10];
    s.pull(-1, a);
    s.publish(-1, a, ring, rring);
    s.pull(0, a);
    s.publish(0, a, ring, rring);
    int r = 0;
    while (true) {
      s.pull(r + 1, b);
      s.publish(r + 1, b, ring, rring);
      __syncthreads();
      s.finish(r, a, ring, rring);
      if (++r >= h) break;
      s.pull(r + 1, a);
      s.publish(r + 1, a, ring, rring);
      __syncthreads();
      s.finish(r, b, ring, rring);
      if (++r >= h) break;
    }
  } else {
    float a[C1][10], b[C1][10], c[C1][10];
    s.pull(-1, a);
    s.publish(-1, a, ring, rring);
    s.pull(0, a);
    s.pull(1, b);
    s.publish(0, a, ring, rring);
    int r = 0;
    // a: row r (published); b: row r + 1 (in flight)
    while (true) {
      if (r + 2 <= h) s.pull(r + 2, c);
      s.publish(r + 1, b, ring, rring);
      __syncthreads();
      s.finish(r, a, ring, rring);
      if (++r >= h) break;
      if (r + 2 <= h) s.pull(r + 2, a);
      s.publish(r + 1, c, ring, rring);
      __syncthreads();
      s.finish(r, b, ring, rring);
      if (++r >= h) break;
      if (r + 2 <= h) s.pull(r + 2, b);
      s.publish(r + 1, a, ring, rring);
      __syncthreads();
      s.finish(r, c, ring, rring);
      if (++r >= h) break;
    }
  }
}

// Work distribution: workgroup b takes items b, b + grid, ... of the table
// (one item each when the grid is as large as the table).
template <class S, int NT, int CPT, int PF>
__global__ __launch_bounds__(NT) void k_step(const InstDesc* __restrict__ descs,
                                             const TileItem* __restrict__ items,
                                             const int* __restrict__ nitems_p, int sub) {
  using St = Strip<S, NT, CPT>;
  __shared__ float ring[4][St::SW + 2];
  const int nitems = *nitems_p;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const TileItem ti = items[__builtin_amdgcn_readfirstlane(it)];
    const InstDesc* __restrict__ dp = descs + __builtin_amdgcn_readfirstlane(ti.inst);
    if (step_runs(dp, sub)) {
      St s;
      s.setup(dp, ti, sub);
      march<St, PF>(s, ring);
      report_unstable(dp, s.bad);
    }
    __syncthreads();  // the next item reuses the ring
  }
}

template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const int (&op)[NV]);

// A step that also records the diagnostics of the state it advances: one
// partial record (kPartialStride doubles, the layout of the separate
// diagnostics pass) per item, folded afterwards in item order.
constexpr int kDiagThreads = 256;
template <class S>
__global__ __launch_bounds__(kDiagThreads) void k_step_diag(const InstDesc* __restrict__ descs,
                                                            const TileItem* __restrict__ items,
                                                            const int* __restrict__ nitems_p,
                                                            int sub, double* __restrict__ partials) {
  using St = Strip<S, kDiagThreads, 1, true>;
  __shared__ float ring[4][St::SW + 2];
  __shared__ double rring[4][St::SW + 2];
  const int nitems = *nitems_p;
  const int op[10] = {0, 0, 0, 0, 0, 1, 0, 0, 1, 2};
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const TileItem ti = items[__builtin_amdgcn_readfirstlane(it)];
    const InstDesc* __restrict__ dp = descs + __builtin_amdgcn_readfirstlane(ti.inst);
    St s;
    s.setup(dp, ti, sub);
    s.diag_zero();
    march<St, 2>(s, ring, rring);
    report_unstable(dp, s.bad);
    block_reduce<10>(s.acc, op);
    if (threadIdx.x == 0)
      for (int q = 0; q < 10; ++q) partials[(size_t)it * kPartialStride + q] = s.acc[q];
    __syncthreads();  // the next item reuses the rings
  }
}

// ============================================================== paired-column step kernel
//
// Wave-local variant of the same step.  Each lane loads one aligned pair of
// adjacent cells per population (32 bits for FP16 storage, 64 for FP32), so a
// wavefront moves twice the bytes per memory instruction.  The pulled values
// shifted by one column come from the neighbouring lane (shuffles) instead of
// misaligned loads, and the psi rows stay in registers: no LDS, no barrier.
// A wavefront covers 128 consecutive columns (mod nx) starting two columns
// left of its 124-column output segment; lanes 0 and 63 only supply the
// halo.  Needs nx even and nx >= 128, so every pair is aligned and a wave
// never wraps onto itself.

constexpr int kPairOut = 124;  // output columns per wavefront

// Whole-wavefront lane shifts (DPP wave_shr:1 / wave_shl:1): lane l receives
// the value of lane l - 1 (from_prev) or l + 1 (from_next); the lane with no
// source (0, resp. 63) receives zero and is a halo lane whose result is not
// used.
__device__ __forceinline__ uint32_t lane_from_prev(uint32_t v) {
  return __builtin_amdgcn_update_dpp(0u, v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t lane_from_next(uint32_t v) {
  return __builtin_amdgcn_update_dpp(0u, v, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ float lane_from_prev(float v) {
  return __builtin_bit_cast(float, lane_from_prev(__builtin_bit_cast(uint32_t, v)));
}
__device__ __forceinline__ float lane_from_next(float v) {
  return __builtin_bit_cast(float, lane_from_next(__builtin_bit_cast(uint32_t, v)));
}

// float(half) + s rounded once, the half taken from the low or the high 16
// bits of w: one mixed-precision FMA (h * 1 + s) instead of a conversion and
// an add.  The product is exact, so the result equals float(h) + s.
__device__ __forceinline__ float half_lo_plus(uint32_t w, float s) {
  float r;
  asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(s));
  return r;
}
__device__ __forceinline__ float half_hi_plus(uint32_t w, float s) {
  float r;
  asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(s));
  return r;
}

// Per-storage access to one lane's pair word: the two cells (lo = left,
// hi = right), the right cell of the previous lane's pair and the left cell
// of the next lane's pair.
template <class S>
struct PairIO;

template <>
struct PairIO<StoreF32> {
  using W = uint64_t;
  __device__ static __forceinline__ float lo(W w, float) {
    return __builtin_bit_cast(float, (uint32_t)w);
  }
  __device__ static __forceinline__ float hi(W w, float) {
    return __builtin_bit_cast(float, (uint32_t)(w >> 32));
  }
  __device__ static __forceinline__ float hi_of_prev(W w, float) {
    return __builtin_bit_cast(float, lane_from_prev((uint32_t)(w >> 32)));
  }
  __device__ static __forceinline__ float lo_of_next(W w, float) {
    return __builtin_bit_cast(float, lane_from_next((uint32_t)w));
  }
  __device__ static __forceinline__ W make(float a, float b, float, float) {
    return (uint64_t)__builtin_bit_cast(uint32_t, a) |
           ((uint64_t)__builtin_bit_cast(uint32_t, b) << 32);
  }
};

template <>
struct PairIO<StoreF16S> {
  using W = uint32_t;
  __device__ static __forceinline__ float lo(W w, float sh) { return half_lo_plus(w, sh); }
  __device__ static __forceinline__ float hi(W w, float sh) { return half_hi_plus(w, sh); }
  __device__ static __forceinline__ float hi_of_prev(W w, float sh) {
    return half_hi_plus(lane_from_prev(w), sh);
  }
  __device__ static __forceinline__ float lo_of_next(W w, float sh) {
    return half_lo_plus(lane_from_next(w), sh);
  }
  __device__ static __forceinline__ W make(float a, float b, float sa, float sb) {
    const uint16_t ha = __builtin_bit_cast(uint16_t, static_cast<_Float16>(a - sa));
    const uint16_t hb = __builtin_bit_cast(uint16_t, static_cast<_Float16>(b - sb));
    return (uint32_t)ha | ((uint32_t)hb << 16);
  }
};

// Per-cell-shift FP16: the reference density q and the stored value h are
// two halves of two words; q * w + h in one mixed-precision FMA (single
// rounding, exactly StoreF16C::decode).  _lo takes the low halves, _hi the
// high halves.
__device__ __forceinline__ float mix_lo(uint32_t q, float w, uint32_t h) {
  float r;
  asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(q), "v"(w), "v"(h));
  return r;
}
// The same on two halves held in registers of their own (the instruction
// reads the low 16 bits only, so they need no masking).
__device__ __forceinline__ float mix_lo(_Float16 q, float w, _Float16 h) {
  float r;
  asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(q), "v"(w), "v"(h));
  return r;
}
__device__ __forceinline__ float mix_hi(uint32_t q, float w, uint32_t h) {
  float r;
  asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[1,0,1] op_sel_hi:[1,0,1]"
      : "=v"(r) : "v"(q), "v"(w), "v"(h));
  return r;
}

template <>
struct PairIO<StoreF16C> {
  using W = uint32_t;
  __device__ static __forceinline__ W pack(_Float16 a, _Float16 b) {
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
  }
};

// psi of one row around a lane's pair (left neighbour, the two cells, right
// neighbour) and the densities of the two cells.
struct PsiRow {
  float l, a, b, r;
  float rho_a, rho_b;
};

template <class S>
struct PairStrip {
  using T = typename S::T;
  using IO = PairIO<S>;
  using W = typename IO::W;
  // words a lane loads per row: the nine populations, plus the reference
  // density of rows y, y - 1, y + 1 for per-cell-shift storage
  static constexpr int kWords = S::kCellShift ? 12 : 9;

  uint64_t src, dst;
  float sh[9];
  int nx, ny, y0, h, dir;
  uint32_t pb;  // byte offset of this lane's pair within a row
  bool out_ok;  // this lane writes its pair
  float G, tau, omega;
  uint64_t bad;  // lanes that collided a cell with a non-finite or non-positive density

  __device__ __forceinline__ static uint64_t uniform(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
  }
  // The lane offset re-materialised where it is used, so that the address is
  // formed as scalar row base + 32-bit lane offset inside the loop body
  // (global_* with saddr) rather than from a hoisted 64-bit vector offset.
  __device__ __forceinline__ uint32_t lane_offset() const {
    uint32_t o = pb;
    asm volatile("" : "+v"(o));
    return o;
  }
  __device__ __forceinline__ gptr<const W> in_pair(int i, int y, uint32_t o) const {
    const uint64_t row = uniform(src + row_index(i, y, nx, ny) * sizeof(T));
    return reinterpret_cast<gptr<const W>>(as_global<const char>(row) + o);
  }
  __device__ __forceinline__ gptr<W> out_pair(int i, int y, uint32_t o) const {
    const uint64_t row = uniform(dst + row_index(i, y, nx, ny) * sizeof(T));
    return reinterpret_cast<gptr<W>>(as_global<char>(row) + o);
  }
  __device__ __forceinline__ gptr<const W> rhat_in_pair(int y, uint32_t o) const {
    const uint64_t row = uniform(src + rhat_row(y, nx, ny) * sizeof(T));
    return reinterpret_cast<gptr<const W>>(as_global<const char>(row) + o);
  }
  __device__ __forceinline__ gptr<W> rhat_out_pair(int y, uint32_t o) const {
    const uint64_t row = uniform(dst + rhat_row(y, nx, ny) * sizeof(T));
    return reinterpret_cast<gptr<W>>(as_global<char>(row) + o);
  }

  __device__ __forceinline__ void setup(const InstDesc* __restrict__ dp, const TileItem& ti, int sub,
                                        int wave, int lane) {
    nx = dp->nx;
    ny = dp->ny;
    y0 = ti.y0;
    h = ti.h;
    dir = ti.dir;
    G = dp->G;
    tau = dp->tau;
    omega = dp->omega;
    const float rho0 = dp->rho0;
    const int par = step_parity(dp, sub);
    const uint64_t a = dp->pop[0], b = dp->pop[1];
    src = par ? b : a;
    dst = par ? a : b;
    const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
#pragma unroll
    for (int i = 0; i < 9; ++i) sh[i] = ws[i] * rho0;
    const int xs = ti.x0 + wave * kPairOut;          // first output column of this wave
    const int wcols = min(kPairOut, nx - xs);        // output columns (even; may be <= 0)
    int c = xs - 2 + 2 * lane;                       // first column of the lane's pair
    c = c < 0 ? c + nx : (c >= nx ? c - nx : c);
    pb = (uint32_t)c * (uint32_t)sizeof(T);
    out_ok = lane >= 1 && lane <= 62 && 2 * (lane - 1) < wcols;
    bad = 0;
  }

  __device__ __forceinline__ int row_of(int j) const {
    int y = dir ? y0 + h - 1 - j : y0 + j;
    return y < 0 ? y + ny : (y >= ny ? y - ny : y);
  }

  // Raw stored pairs feeding row j: population i comes from row y - e_iy.
  __device__ __forceinline__ void load(int j, W (&w)[kWords]) const {
    const int y = row_of(j);
    const int ym = wrap_dec(y, ny), yp = wrap_inc(y, ny);
    const uint32_t o = lane_offset();
    w[0] = *in_pair(0, y, o);
    w[1] = *in_pair(1, y, o);
    w[2] = *in_pair(2, ym, o);
    w[3] = *in_pair(3, y, o);
    w[4] = *in_pair(4, yp, o);
    w[5] = *in_pair(5, ym, o);
    w[6] = *in_pair(6, ym, o);
    w[7] = *in_pair(7, yp, o);
    w[8] = *in_pair(8, yp, o);
    if constexpr (S::kCellShift) {
      w[9] = *rhat_in_pair(y, o);
      w[10] = *rhat_in_pair(ym, o);
      w[11] = *rhat_in_pair(yp, o);
    }
  }

  // Pre-collision populations of the pair's two cells and the row's psi.
  // Populations pulled from x - 1 (e_ix = +1: 1, 5, 8) take the previous
  // lane's upper cell for cell a; those pulled from x + 1 (e_ix = -1: 3, 6, 7)
  // take the next lane's lower cell for cell b.
  __device__ __forceinline__ void expand(const W (&w)[kWords], float (&fa)[9], float (&fb)[9],
                                         PsiRow& ps) const {
    if constexpr (S::kCellShift) {
      // each value with the reference density of the cell it was read from
      const W qy = w[9], qm = w[10], qp = w[11];
      const W pqy = lane_from_prev(qy), pqm = lane_from_prev(qm), pqp = lane_from_prev(qp);
      const W nqy = lane_from_next(qy), nqm = lane_from_next(qm), nqp = lane_from_next(qp);
      fa[0] = mix_lo(qy, kW0, w[0]);
      fb[0] = mix_hi(qy, kW0, w[0]);
      fa[2] = mix_lo(qm, kW1, w[2]);
      fb[2] = mix_hi(qm, kW1, w[2]);
      fa[4] = mix_lo(qp, kW1, w[4]);
      fb[4] = mix_hi(qp, kW1, w[4]);
      fa[1] = mix_hi(pqy, kW1, lane_from_prev(w[1]));
      fb[1] = mix_lo(qy, kW1, w[1]);
      fa[5] = mix_hi(pqm, kW2, lane_from_prev(w[5]));
      fb[5] = mix_lo(qm, kW2, w[5]);
      fa[8] = mix_hi(pqp, kW2, lane_from_prev(w[8]));
      fb[8] = mix_lo(qp, kW2, w[8]);
      fa[3] = mix_hi(qy, kW1, w[3]);
      fb[3] = mix_lo(nqy, kW1, lane_from_next(w[3]));
      fa[6] = mix_hi(qm, kW2, w[6]);
      fb[6] = mix_lo(nqm, kW2, lane_from_next(w[6]));
      fa[7] = mix_hi(qp, kW2, w[7]);
      fb[7] = mix_lo(nqp, kW2, lane_from_next(w[7]));
    } else {
      fa[0] = IO::lo(w[0], sh[0]);
      fb[0] = IO::hi(w[0], sh[0]);
      fa[2] = IO::lo(w[2], sh[2]);
      fb[2] = IO::hi(w[2], sh[2]);
      fa[4] = IO::lo(w[4], sh[4]);
      fb[4] = IO::hi(w[4], sh[4]);
      fa[1] = IO::hi_of_prev(w[1], sh[1]);
      fb[1] = IO::lo(w[1], sh[1]);
      fa[5] = IO::hi_of_prev(w[5], sh[5]);
      fb[5] = IO::lo(w[5], sh[5]);
      fa[8] = IO::hi_of_prev(w[8], sh[8]);
      fb[8] = IO::lo(w[8], sh[8]);
      fa[3] = IO::hi(w[3], sh[3]);
      fb[3] = IO::lo_of_next(w[3], sh[3]);
      fa[6] = IO::hi(w[6], sh[6]);
      fb[6] = IO::lo_of_next(w[6], sh[6]);
      fa[7] = IO::hi(w[7], sh[7]);
      fb[7] = IO::lo_of_next(w[7], sh[7]);
    }
    ps.rho_a = density(fa);
    ps.rho_b = density(fb);
    ps.a = psi_of(ps.rho_a);
    ps.b = psi_of(ps.rho_b);
    ps.l = lane_from_prev(ps.b);
    ps.r = lane_from_next(ps.a);
  }

  // Collide the pair at march position r and store it.  Marching upwards the
  // previous position is the row above.
  __device__ __forceinline__ void finish(int r, float (&fa)[9], float (&fb)[9], const PsiRow& prev,
                                         const PsiRow& md, const PsiRow& next) {
    const PsiRow& dn = dir ? next : prev;
    const PsiRow& up = dir ? prev : next;
    float Fx, Fy;
    force_of(md.a, md.b, up.a, md.l, dn.a, up.b, up.l, dn.l, dn.b, G, Fx, Fy);
    bad |= unstable_lanes(md.rho_a, out_ok) | unstable_lanes(md.rho_b, out_ok);
    collide(fa, md.rho_a, Fx, Fy, tau, omega);
    force_of(md.b, md.r, up.b, md.a, dn.b, up.r, up.a, dn.a, dn.r, G, Fx, Fy);
    collide(fb, md.rho_b, Fx, Fy, tau, omega);
    if (out_ok) {
      const int y = row_of(r);
      const uint32_t o = lane_offset();
      if constexpr (S::kCellShift) {
        const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
        const T ra = S::ref(md.rho_a), rb = S::ref(md.rho_b);
#pragma unroll
        for (int i = 0; i < 9; ++i)
          *out_pair(i, y, o) = IO::pack(S::encode(fa[i], ra, ws[i]), S::encode(fb[i], rb, ws[i]));
        *rhat_out_pair(y, o) = IO::pack(ra, rb);
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          const W v = IO::make(fa[i], fb[i], sh[i], sh[i]);
          if constexpr (S::kStream)
            __builtin_nontemporal_store(v, out_pair(i, y, o));
          else
            *out_pair(i, y, o) = v;
        }
      }
    }
  }
};

template <class S, int NW, int PF>
__global__ __launch_bounds__(64 * NW) void k_step_pair(const InstDesc* __restrict__ descs,
                                                       const TileItem* __restrict__ items,
                                                       const int* __restrict__ nitems_p, int sub) {
  using St = PairStrip<S>;
  using W = typename St::W;
  const int nitems = *nitems_p;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const TileItem ti = items[__builtin_amdgcn_readfirstlane(it)];
    const InstDesc* __restrict__ dp = descs + __builtin_amdgcn_readfirstlane(ti.inst);
    if (step_runs(dp, sub) && ti.x0 + wave * kPairOut < dp->nx) {
      St s;
      s.setup(dp, ti, sub, wave, lane);
      const int h = s.h;
      W w0[St::kWords], w1[St::kWords];
      float fa0[9], fb0[9], fa1[9], fb1[9];
      PsiRow p0, p1, p2;
      s.load(-1, w0);
      s.expand(w0, fa0, fb0, p0);  // halo row: psi only
      s.load(0, w0);
      if constexpr (PF == 2) s.load(1, w1);
      s.expand(w0, fa0, fb0, p1);
      // One march position: the row r held in (fa, fb) with psi pm is
      // collided once the next row (into (fn, gn), psi pn) is expanded.
      // The roles rotate with period 2 for the populations and 3 for the
      // psi rows, so six positions per turn need no register copies.
      int r = 0;
      auto pos = [&](float(&fa)[9], float(&fb)[9], float(&fn)[9], float(&gn)[9],
                     W(&wn)[St::kWords], W(&wl)[St::kWords], PsiRow& pp, PsiRow& pm,
                     PsiRow& pn) -> bool {
        if constexpr (PF == 2) {
          // wn: loads of row r + 1 already in flight; wl: free for row r + 2
          if (r + 2 <= h) s.load(r + 2, wl);
          s.expand(wn, fn, gn, pn);
        } else {
          s.load(r + 1, wn);
          s.expand(wn, fn, gn, pn);
        }
        s.finish(r, fa, fb, pp, pm, pn);
        return ++r >= h;
      };
      while (true) {
        if (pos(fa0, fb0, fa1, fb1, w1, w0, p0, p1, p2)) break;
        if (pos(fa1, fb1, fa0, fb0, w0, w1, p1, p2, p0)) break;
        if (pos(fa0, fb0, fa1, fb1, w1, w0, p2, p0, p1)) break;
        if (pos(fa1, fb1, fa0, fb0, w0, w1, p0, p1, p2)) break;
        if (pos(fa0, fb0, fa1, fb1, w1, w0, p1, p2, p0)) break;
        if (pos(fa1, fb1, fa0, fb0, w0, w1, p2, p0, p1)) break;
      }
      report_unstable(dp, s.bad);
    }
  }
}

// ============================================================== two fused time steps
//
// Temporal blocking: a workgroup advances its strip of a band by two time
// steps in one pass, so the populations cross HBM once per two updates.  The
// post-collision values of the intermediate step never leave the CU: they go
// through a three-row LDS ring, rounded through the storage form exactly as a
// store and a load would round them, so the result is bitwise that of two
// single steps.  Strip slot k (see strip_slot) holds column x0 - 3 + k (mod
// nx).  Per march row j:
//   1. pull f(t) of row j + 3 (loads issued PF rows ahead), publish psi(t);
//   2. collide row j + 2 into the ring (slots 1 .. NT - 2);
//   3. pull f(t + 1) of row j + 1 from the ring, publish psi(t + 1);
//   4. collide row j and store it (columns x0 .. x0 + W - 1).
// One barrier separates each stage from the next.  The band's rows are
// reached through three halo rows above and below; a strip writes W <= NT - 6
// columns.
//
// Moment storage keeps a record per cell (the values it wrote, as mass,
// momentum and six half-precision deviations), so stage 1 is split in two:
// each thread loads and decodes the record of its own column of row j + 4
// into a fourth LDS ring, and after a barrier pulls f(t) of row j + 3 from
// that ring.  The pull costs one more halo column per side (slot k holds
// column x0 - 4 + k, W <= NT - 8) and one more halo row above and below.

template <class S>
struct RawCell {
  typename S::T v[9];
  typename S::T q[9];  // reference densities (per-cell-shift storage)
};

// A moment record as loaded: mass, momentum and the six deviations.
struct RawRec {
  float r[3];
  _Float16 h[6];
};

// Halo columns on each side of a two-step strip.
template <class S>
constexpr int fused_halo() {
  return S::kMoment ? 4 : 3;
}

// Strip slot of this thread: slot k holds column x0 - H + k (H halo columns
// per side) and is the thread's index in the LDS rings.  In FP32 thread t
// takes slot t + H (mod NT), so lane t loads and stores column x0 + t and a
// wavefront's accesses start on the strip's (aligned) first column; the last
// H threads take the left halo.  (2-3% faster in FP32, 1-2% slower in the
// FP16 forms, which keep slot t.)
template <class S, int NT, int H = fused_halo<S>()>
__device__ __forceinline__ int strip_slot() {
  static_assert((NT & (NT - 1)) == 0, "NT is a power of two");
  constexpr int kShift = std::is_same<S, StoreF32>::value ? H : 0;
  return ((int)threadIdx.x + kShift) & (NT - 1);
}

template <class S, int NT, int PF, int W, int H = fused_halo<S>()>
struct Fused2 {
  static constexpr int kH = H;
  static_assert(W <= NT - 2 * kH, "kH halo lanes on each side");
  using T = typename S::T;

  static_assert(SCLBM_ROW_LAYOUT, "lattice row y keeps its nine population rows together");

  uint64_t src, dst;    // population arrays read and written
  uint64_t qsrc, qdst;  // their reference-density planes (per-cell shift)
  float sh[9];
  float one;  // 1.0, opaque to the compiler (opaque_one)
  int nx, ny, y0, h, dir, wcols;
  uint32_t lrow, prow;  // bytes of a lattice row (nine population rows) and of one population row
  uint32_t bc, bm, bp;  // byte offsets of this thread's column and its neighbours
  uint32_t bc4;         // byte offset of this thread's column in an FP32 row
  bool out;             // this thread stores a cell of the second step
  bool wrap;            // the grid is one periodic strip (nx <= NT)
  float G, tau, omega;

  __device__ __forceinline__ static uint64_t uniform(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
  }
  __device__ __forceinline__ static uint32_t fresh(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
  }
  // Buffer resource over `bytes` bytes from base + y * pitch (one population
  // row of lattice row y when base is the population's row 0).
  __device__ __forceinline__ static __amdgpu_buffer_rsrc_t rows(uint64_t base, int y,
                                                               uint32_t pitch, uint32_t bytes) {
    const uint64_t a = uniform(base + (uint64_t)(uint32_t)y * pitch);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(a), (short)0, (int)bytes,
                                             0x00020000);
  }
  // Load at byte `off` of the row that starts at the (wave-uniform) address row.
  __device__ __forceinline__ static T ld(uint64_t row, uint32_t off) {
    return *reinterpret_cast<gptr<const T>>(reinterpret_cast<gptr<const char>>(uniform(row)) + off);
  }

  __device__ __forceinline__ void setup(const InstDesc* __restrict__ dp, const TileItem& ti,
                                        int sub) {
    nx = dp->nx;
    ny = dp->ny;
    y0 = ti.y0;
    h = ti.h;
    dir = ti.dir;
    wcols = min(W, nx - ti.x0);
    G = dp->G;
    tau = dp->tau;
    omega = dp->omega;
    const float rho0 = dp->rho0;
    const int par = pair_parity(dp, sub);
    const uint64_t a = dp->pop[0], b = dp->pop[1];
    src = par ? b : a;
    dst = par ? a : b;
    qsrc = src + rhat_row(0, nx, ny) * sizeof(T);
    qdst = dst + rhat_row(0, nx, ny) * sizeof(T);
    prow = (uint32_t)nx * (uint32_t)sizeof(T);
    lrow = 9u * prow;
    const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
#pragma unroll
    for (int i = 0; i < 9; ++i) sh[i] = ws[i] * rho0;
    one = opaque_one();
    const int t = strip_slot<S, NT, kH>();
    int c = (ti.x0 - kH + t) % nx;
    c = c < 0 ? c + nx : c;
    bc = (uint32_t)c * (uint32_t)sizeof(T);
    bc4 = (uint32_t)c * 4u;
    bm = (uint32_t)wrap_dec(c, nx) * (uint32_t)sizeof(T);
    bp = (uint32_t)wrap_inc(c, nx) * (uint32_t)sizeof(T);
    // A grid no wider than the workgroup is marched as one periodic strip
    // (x0 = 0): ring column x < nx holds lattice column (x - kH) mod nx, the
    // ring's neighbours wrap at nx, and every column is written.
    wrap = nx <= NT;
    out = wrap ? t < nx : (t >= kH && t - kH < wcols);
  }

  // Lattice row of march position j (any j in [-kH, h + kH - 1]).  As
  // y0 + h <= ny the unwrapped row lies in [-kH, ny + kH - 1]: one wrap maps
  // it into the grid once ny >= kH; below that (ny = 1 or 2 for kH = 3, the
  // low bits) the remainder.
  __device__ __forceinline__ int row_of(int j) const {
    const int y = dir ? y0 + h - 1 - j : y0 + j;
    const int w = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    if constexpr (kH > 3)
      return ny < kH ? ((y % ny) + ny) % ny : w;
    else
      return ny < 3 ? (y & (ny - 1)) : w;
  }

  // Moment storage: issues the loads of the record of this thread's column
  // in row j (mass, momentum, six deviations).
  __device__ __forceinline__ void fetch_record(int j, RawRec& r) const {
    const int y = row_of(j);
    const uint64_t b = src + mom_row(y, nx);
    const uint32_t c2 = fresh(bc), c4 = fresh(bc4);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      r.r[k] = *reinterpret_cast<gptr<const float>>(
          reinterpret_cast<gptr<const char>>(uniform(b + mom_f32(k, nx))) + c4);
#pragma unroll
    for (int i = 3; i < 9; ++i) r.h[i - 3] = ld(b + mom_f16(i, nx), c2);
  }

  // Issues the loads of row j's pulled populations (f_i(x) = A_i(x - e_i))
  // into v, and for per-cell-shift storage the reference densities of the
  // cells they come from into q.
  __device__ __forceinline__ void fetch(int j, T* v, T* q) const {
    const int y = row_of(j);
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const uint32_t c = fresh(bc), m = fresh(bm), p = fresh(bp);
    const uint64_t r0 = src + (uint64_t)(uint32_t)y * lrow, rm = src + (uint64_t)(uint32_t)ym * lrow,
                   rp = src + (uint64_t)(uint32_t)yp * lrow;
    v[0] = ld(r0, c);
    v[1] = ld(r0 + prow, m);
    v[2] = ld(rm + 2 * prow, c);
    v[3] = ld(r0 + 3 * prow, p);
    v[4] = ld(rp + 4 * prow, c);
    v[5] = ld(rm + 5 * prow, m);
    v[6] = ld(rm + 6 * prow, p);
    v[7] = ld(rp + 7 * prow, p);
    v[8] = ld(rp + 8 * prow, m);
    if constexpr (S::kCellShift) {
      const uint64_t q0 = qsrc + (uint64_t)(uint32_t)y * prow,
                     qm = qsrc + (uint64_t)(uint32_t)ym * prow,
                     qp = qsrc + (uint64_t)(uint32_t)yp * prow;
      q[0] = ld(q0, c);
      q[1] = ld(q0, m);
      q[2] = ld(qm, c);
      q[3] = ld(q0, p);
      q[4] = ld(qp, c);
      q[5] = ld(qm, m);
      q[6] = ld(qm, p);
      q[7] = ld(qp, p);
      q[8] = ld(qp, m);
    }
  }

  // Widening of the pulled values, as the storage type reads them back: one
  // mixed-precision FMA per value.  Per-cell-shift storage: rhohat * w_i + h,
  // both halves read directly, equal to StoreF16C::decode.  FP16-shifted:
  // h * 1 + w_i rho0, equal to StoreF16S::load (the 1 is opaque to the
  // compiler, which otherwise turns the FMA into a conversion and an add).
  __device__ __forceinline__ void decode(const RawCell<S>& r, float (&f)[10]) const {
    const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if constexpr (S::kCellShift)
        f[i] = mix_lo(r.q[i], ws[i], r.v[i]);
      else
        f[i] = widen(r.v[i], sh[i]);
    }
    f[9] = density(f);
  }

  // An FP16-shifted value read back: float(h) + shift in one mixed FMA.
  __device__ __forceinline__ float widen(T h, float shift) const {
    return fmaf(static_cast<float>(h), one, shift);
  }

  // Moment storage: the nine values a collided cell's record reads back as
  // (its mass rho, the momentum of v and the six deviations, decoded).
  __device__ __forceinline__ static void through_record(const float (&v)[10], float rho,
                                                        float (&g)[9]) {
    float jx, jy;
    _Float16 h[6];
    mom_encode(v, rho, jx, jy, h);
    mom_decode(rho, jx, jy, h, g);
  }

  // A post-collision value as the next step would read it back from storage.
  __device__ __forceinline__ float through_storage(float v, int i, float rho) const {
    const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
    if constexpr (S::kCellShift) {
      const T rh = S::ref(rho);
      return mix_lo(rh, ws[i], S::encode(v, rh, ws[i]));
    } else if constexpr (sizeof(T) == 2) {
      return widen(S::pack(v, sh[i]), sh[i]);
    } else {
      return v;  // FP32 stores the value itself
    }
  }

  // Stores of a row go through buffer resources with the row as its range:
  // lanes that own no output column pass an offset past the end, and the
  // hardware drops those stores.  No branch around the stores, so the wait
  // counts before the next loads stay exact (loads issued before a
  // branch-skipped store block would otherwise be waited for with the stores).
  // (One resource for the nine rows with the population's row as a scalar
  // offset takes fewer scalar instructions but ran 2% slower in FP32.)
  __device__ __forceinline__ static void put(__amdgpu_buffer_rsrc_t r, uint32_t off, T v) {
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0,
                                            S::kStream ? 2 : 0);  // 2: non-temporal
    else
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, (int)off, 0, 0);
  }

  __device__ __forceinline__ void store(int j, const float (&f)[10]) const {
    const int y = row_of(j);
    const uint32_t c = out ? fresh(bc) : 0x80000000u;
    if constexpr (S::kMoment) {
      // the record: the density the cell collided with (its mass), the
      // momentum of the collided values and the six deviations
      float jx, jy;
      _Float16 hv[6];
      mom_encode(f, f[9], jx, jy, hv);
      const uint32_t c4 = out ? fresh(bc4) : 0x80000000u;
      const uint32_t pitch = 24u * (uint32_t)nx;
      const float r3[3] = {f[9], jx, jy};
#pragma unroll
      for (int k = 0; k < 3; ++k)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, r3[k]),
                                              rows(dst + mom_f32(k, nx), y, pitch, 4u * nx),
                                              (int)c4, 0, 0);
#pragma unroll
      for (int i = 3; i < 9; ++i)
        put(rows(dst + mom_f16(i, nx), y, pitch, 2u * nx), c, hv[i - 3]);
    } else if constexpr (S::kCellShift) {
      const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
      const T rh = S::ref(f[9]);
#pragma unroll
      for (int i = 0; i < 9; ++i) put(rows(dst + i * prow, y, lrow, prow), c, S::encode(f[i], rh, ws[i]));
      put(rows(qdst, y, prow, prow), c, rh);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) put(rows(dst + i * prow, y, lrow, prow), c, S::pack(f[i], sh[i]));
    }
  }
};

// Interaction force at ring column t from three psi ring rows: dn holds row
// y - 1, md row y, up row y + 1; l and r are the ring columns left and right
// of t.
__device__ __forceinline__ void ring_force(const float* dn, const float* md, const float* up, int t,
                                           int l, int r, float G, float& Fx, float& Fy) {
  force_of(md[t], md[r], up[t], md[l], dn[t], up[r], up[l], dn[l], dn[r], G, Fx, Fy);
}

// Ring slot of march row r >= -9 in a ring of three rows, and of row r >= -10
// in a ring of two.
__device__ __forceinline__ int slot3(int r) { return (r + 9) % 3; }
__device__ __forceinline__ int slot2(int r) { return (r + 10) & 1; }

// Calls fn(integral_constant<int, I>) for I = 0, 1, ... in order.
template <class Fn, int... I>
__device__ __forceinline__ void unrolled(std::integer_sequence<int, I...>, Fn&& fn) {
  (fn(std::integral_constant<int, I>{}), ...);
}

// The march of the two-step kernels.  DIAG = true also accumulates the FP64
// diagnostics of the state the launch reads (the cells the workgroup owns,
// from the populations pulled for the first step, per cell in the arithmetic
// of the separate pass; FP64 rho goes through a third LDS ring) and writes
// one partial record per item.
template <class S, int NT, int PF, int W, bool DIAG>
__device__ __forceinline__ void two_step_march(const InstDesc* __restrict__ descs,
                                               const TileItem* __restrict__ items,
                                               const int* __restrict__ nitems_p, int sub,
                                               double* __restrict__ partials) {
  static_assert(PF == 1 || PF == 2, "one or two rows of loads in flight");
  using F = Fused2<S, NT, PF, W>;
  using T = typename S::T;
  // FP32 rows are loaded straight into the registers they are collided in:
  // a slot lives from its loads to the first collision, PF + 2 positions.
  // Half-precision rows land in PF + 1 raw slots and are widened into two
  // rotating FP32 rows.  The loads of a position always go to a slot that is
  // idle at that point.  The march is unrolled over U positions, a multiple
  // of every rotation period, so each slot stays in fixed registers.
  constexpr bool kInPlace = std::is_same<S, StoreF32>::value;
  constexpr int NR = kInPlace ? PF + 2 : PF + 1;
  // With U a multiple of 3 the LDS ring slots are constants too (not taken
  // for the diagnostics variant, whose longer period needs too many
  // registers).
  constexpr int U = !DIAG && (NR == 2 || NR == 3)
                        ? 6
                        : (NR % 2 == 0 ? NR : 2 * NR);
  constexpr bool kFixedRing = U % 3 == 0;
  constexpr int NF = kInPlace ? NR : 2;  // FP32 rows of the first step
  __shared__ float psa[3][NT];  // psi(t) rows
  __shared__ float psb[3][NT];  // psi(t + 1) rows
  // f*(t + 1) of the rows that the pull of row j + 1 reads, as read back from
  // storage, each population kept only until it is read.  Populations 0, 1
  // and 3 come from row j + 1 itself, written one position earlier (two
  // slots).  Of the rows on either side, the one written at this position
  // (row j + 2) is read at once (one slot) and the one written two positions
  // earlier (row j) is read last (three slots); which three populations each
  // side supplies follows the march direction.  18 rows of NT values instead
  // of 27, which lets more workgroups share a CU's LDS.
  __shared__ float fmd[2][3][NT];   // populations 0, 1, 3
  __shared__ float fnew[3][NT];     // row j + 2: the side it lies on
  __shared__ float fold[3][3][NT];  // row j: the other side
  __shared__ double rr[DIAG ? 3 : 1][DIAG ? NT : 1];  // FP64 rho(t) rows
  // Moment storage: the decoded records A_i of the rows that the pull of row
  // j + 3 reads, kept by the same rule as the f*(t + 1) rings (row j + 4 is
  // the newest, row j + 2 the oldest).
  constexpr bool kM = S::kMoment;
  __shared__ float amd[kM ? 2 : 1][3][kM ? NT : 1];   // populations 0, 1, 3
  __shared__ float anew[3][kM ? NT : 1];              // row j + 4: the side it lies on
  __shared__ float aold[kM ? 3 : 1][3][kM ? NT : 1];  // row j + 2: the other side
  constexpr int D = fused_halo<S>();  // the march reads rows -D .. h + D - 1
  const int nitems = *nitems_p;
  const int t = strip_slot<S, NT>();  // LDS ring index
  // Columns each stage is valid for: a strip loses one halo column per side
  // to every stencil (moment storage: one more, to the pull of stage 1).
  // Lanes that store nothing still run the last collision (on clamped ring
  // columns) so that the row's stores need no branch.
  constexpr int e = kM ? 1 : 0;
  const bool strip_a = t >= 1 + e && t <= NT - 2 - e;
  const bool strip_b = t >= 2 + e && t <= NT - 3 - e;
  const int strip_f = min(max(t, 1), NT - 2);
  const int op[10] = {0, 0, 0, 0, 0, 1, 0, 0, 1, 2};  // sum, max, min
  (void)op;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const TileItem ti = items[__builtin_amdgcn_readfirstlane(it)];
    const InstDesc* __restrict__ dp = descs + __builtin_amdgcn_readfirstlane(ti.inst);
    double acc[10];
    if constexpr (DIAG) diag_zero(acc);
    if (pair_runs(dp, sub)) {
      F s;
      s.setup(dp, ti, sub);
      const int h = s.h;
      uint64_t bad = 0;  // lanes that collided a cell with a non-finite or non-positive density
      // With constant ring slots the march is instantiated per direction, so
      // that every ring access is the lane's LDS address plus a constant.  In
      // march order the row below a row (y - 1) is the previous one when
      // marching downwards and the next one when marching upwards.
      auto march = [&](auto upward, auto wrap_c) {
      const int below = upward ? 1 : -1;
      // A periodic strip loses no column to the stencils: its lanes t >= nx
      // only decode, and tl and tr, the ring neighbours of column t, wrap at
      // nx.  (Instantiated apart from the plain strip, whose code it would
      // otherwise change.)
      constexpr bool kW = decltype(wrap_c)::value;
      const int nx = s.nx;
      const bool stage_a = kW ? t < nx : strip_a;
      const bool stage_b = kW ? t < nx : strip_b;
      const int tl = kW ? (t == 0 ? nx - 1 : t - 1) : t - 1;
      const int tr = kW ? (t == nx - 1 ? 0 : min(t + 1, NT - 1)) : t + 1;
      const int tf = kW ? t : strip_f;
      const int tfl = kW ? tl : tf - 1, tfr = kW ? tr : tf + 1;
      // (moment storage) ring neighbours of the stage-1 pull, clamped into
      // the ring for the edge lanes, whose pull is not used
      const int tal = kW ? tl : max(t - 1, 0), tar = kW ? tr : min(t + 1, NT - 1);
      using Raw = std::conditional_t<kM, RawRec, RawCell<S>>;
      Raw raw[kInPlace ? 1 : NR];
      float fa[NF][10], fb[2][10];
      // Row R (>= -D) of the first step (moment storage: record row R) is
      // loaded into slot R mod NR.
      auto fetch_row = [&](int row, auto slot_c) {
        constexpr int k = decltype(slot_c)::value;
        if constexpr (kInPlace)
          s.fetch(row, fa[k], nullptr);
        else if constexpr (kM)
          s.fetch_record(row, raw[k]);
        else
          s.fetch(row, raw[k].v, raw[k].q);
      };
      unrolled(std::make_integer_sequence<int, PF>{}, [&](auto k) {
        fetch_row(-D + decltype(k)::value,
                  std::integral_constant<int, (decltype(k)::value + D * NR - D) % NR>{});
      });
      // March position j with phase u = j mod U: issue the loads of row
      // j + D + PF (the band's last row again past its end); decode row j + 3
      // (moment storage: decode record row j + 4 into the record ring, then
      // pull row j + 3 from it) and publish psi(t); collide row j + 2 into the
      // ring; pull f(t + 1) of row j + 1 and publish psi(t + 1); collide row j
      // and store it.
      auto pos = [&](auto lead_c, auto u_c, int j) {
        constexpr bool kLead = decltype(lead_c)::value;  // j < 0: no output row yet
        constexpr int u = decltype(u_c)::value;
        constexpr int kd = (u + D) % NR;  // slot of row j + D
        // ring slot of row j + d (j = u mod U)
        auto ring = [&](int d) { return kFixedRing ? (u + d + 9) % 3 : slot3(j + d); };
        auto ring2 = [&](int d) { return kFixedRing ? (u + d + 10) % 2 : slot2(j + d); };
        float(&fa_c)[10] = fa[kInPlace ? kd : (u + 3) & 1];
        float(&fa_p)[10] = fa[kInPlace ? (u + 2) % NR : (u + 2) & 1];
        float(&fb_c)[10] = fb[(u + 1) & 1];
        float(&fb_p)[10] = fb[u & 1];
        fetch_row(min(j + D + PF, h + D - 1), std::integral_constant<int, (u + D + PF) % NR>{});
        if constexpr (kM) {
          // record row j + 4: its nine values, by the side each is pulled to
          {
            float a[9];
            mom_decode(raw[kd].r[0], raw[kd].r[1], raw[kd].r[2], raw[kd].h, a);
            float(*md)[NT] = amd[ring2(4)];
            float(*old)[NT] = aold[ring(4)];
            float(*dn)[NT] = upward ? anew : old;
            float(*up)[NT] = upward ? old : anew;
            md[0][t] = a[0];
            md[1][t] = a[1];
            md[2][t] = a[3];
            dn[0][t] = a[2];
            dn[1][t] = a[5];
            dn[2][t] = a[6];
            up[0][t] = a[4];
            up[1][t] = a[7];
            up[2][t] = a[8];
          }
          __syncthreads();
          if (!kLead || j >= -6) {  // row j + 3: f_i(x) = A_i(x - e_i)
            const float(*md)[NT] = amd[ring2(3)];
            const float(*old)[NT] = aold[ring(2)];
            const float(*dn)[NT] = upward ? anew : old;
            const float(*up)[NT] = upward ? old : anew;
            fa_c[0] = md[0][t];
            fa_c[1] = md[1][tal];
            fa_c[2] = dn[0][t];
            fa_c[3] = md[2][tar];
            fa_c[4] = up[0][t];
            fa_c[5] = dn[1][tal];
            fa_c[6] = dn[2][tar];
            fa_c[7] = up[1][tar];
            fa_c[8] = up[2][tal];
            fa_c[9] = density(fa_c);
            psa[ring(3)][t] = psi_of(fa_c[9]);
          }
        } else {
          if constexpr (kInPlace)
            fa_c[9] = density(fa_c);
          else
            s.decode(raw[kd], fa_c);
          psa[ring(3)][t] = psi_of(fa_c[9]);
          if constexpr (DIAG) rr[ring(3)][t] = density64(fa_c);
        }
        __syncthreads();
        if constexpr (DIAG) {  // the state read, row j + 2, before its collision
          if ((unsigned)(j + 2) < (unsigned)h && s.out)
            diag_cell(acc, fa_p, t, tl, tr, rr[ring(2 + below)], rr[ring(2)], rr[ring(2 - below)]);
        }
        if ((!kLead || j >= -4) && stage_a) {  // row j + 2
          float Fx, Fy;
          ring_force(psa[ring(2 + below)], psa[ring(2)], psa[ring(2 - below)], t, tl, tr, s.G, Fx,
                     Fy);
          const float rho = fa_p[9];
          collide(fa_p, rho, Fx, Fy, s.tau, s.omega);
          float g[9];
          if constexpr (kM) {
            F::through_record(fa_p, rho, g);
          } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) g[i] = s.through_storage(fa_p[i], i, rho);
          }
          // Row j + 2 is the row below row j + 1 (populations 2, 5, 6 are
          // pulled from it) when marching upwards, the row above it
          // (populations 4, 7, 8) when marching downwards.
          float(*md)[NT] = fmd[ring2(2)];
          float(*old)[NT] = fold[ring(2)];
          float(*dn)[NT] = upward ? fnew : old;
          float(*up)[NT] = upward ? old : fnew;
          md[0][t] = g[0];
          md[1][t] = g[1];
          md[2][t] = g[3];
          dn[0][t] = g[2];
          dn[1][t] = g[5];
          dn[2][t] = g[6];
          up[0][t] = g[4];
          up[1][t] = g[7];
          up[2][t] = g[8];
        }
        __syncthreads();
        if ((!kLead || j >= -2) && stage_b) {
          // row j + 1: f_i(x) = f*_i(x - e_i), rows below feed e_iy = +1
          // (row j is the one written two positions ago)
          const float(*md)[NT] = fmd[ring2(1)];
          const float(*old)[NT] = fold[ring(0)];
          const float(*dn)[NT] = upward ? fnew : old;
          const float(*up)[NT] = upward ? old : fnew;
          fb_c[0] = md[0][t];
          fb_c[1] = md[1][tl];
          fb_c[2] = dn[0][t];
          fb_c[3] = md[2][tr];
          fb_c[4] = up[0][t];
          fb_c[5] = dn[1][tl];
          fb_c[6] = dn[2][tr];
          fb_c[7] = up[1][tr];
          fb_c[8] = up[2][tl];
          fb_c[9] = density(fb_c);
          psb[ring(1)][t] = psi_of(fb_c[9]);
        }
        __syncthreads();
        if constexpr (!kLead) {
          float Fx, Fy;
          ring_force(psb[ring(below)], psb[ring(0)], psb[ring(-below)], tf, tfl, tfr, s.G, Fx, Fy);
          bad |= unstable_lanes(fb_p[9], s.out);
          collide(fb_p, fb_p[9], Fx, Fy, s.tau, s.omega);
          s.store(j, fb_p);
        }
      };
      // 2 D lead-in positions, j = -2 D .. -1
      unrolled(std::make_integer_sequence<int, 2 * D>{}, [&](auto k) {
        constexpr int j = decltype(k)::value - 2 * D;
        pos(std::true_type{}, std::integral_constant<int, (j % U + U) % U>{}, j);
      });
      const auto phases = std::make_integer_sequence<int, U>{};
      int j0 = 0;
      for (; j0 + U <= h; j0 += U)
        unrolled(phases, [&](auto u) { pos(std::false_type{}, u, j0 + decltype(u)::value); });
      unrolled(std::make_integer_sequence<int, U - 1>{}, [&](auto u) {
        if (j0 + decltype(u)::value < h) pos(std::false_type{}, u, j0 + decltype(u)::value);
      });
      };
      auto go = [&](auto wrap_c) {
        if constexpr (!kFixedRing)
          march(s.dir != 0, wrap_c);
        else if (s.dir)
          march(std::true_type{}, wrap_c);
        else
          march(std::false_type{}, wrap_c);
      };
      if (s.wrap)
        go(std::true_type{});
      else
        go(std::false_type{});
      report_unstable(dp, bad);
    }
    if constexpr (DIAG) {
      block_reduce<10>(acc, op);
      if (threadIdx.x == 0)
        for (int q = 0; q < 10; ++q) partials[(size_t)it * kPartialStride + q] = acc[q];
    }
    __syncthreads();  // the next item reuses the rings
  }
}

// W output columns per workgroup (at most NT - kFusedHalo): with W a
// multiple of 16, every strip of an FP32 row starts and ends on a 64-byte
// boundary, so no write granule is shared by two workgroups.
//
// Per-cell-shift storage with one row of loads in flight is compiled for at
// least four wavefronts per SIMD: it fits in 128 VGPRs without spilling
// (unbounded, the compiler takes 133 and the CU holds three).
template <class S, int PF>
constexpr int step2_min_waves() {
  return S::kCellShift && PF == 1 ? 4 : 1;
}
template <class S, int NT, int PF, int W>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(step2_min_waves<S, PF>())))
void k_step2(const InstDesc* __restrict__ descs,
                                              const TileItem* __restrict__ items,
                                              const int* __restrict__ nitems_p, int sub) {
  two_step_march<S, NT, PF, W, false>(descs, items, nitems_p, sub, nullptr);
}

// ============================================================== K fused time steps
//
// FP32 storage, K >= 3 time steps per launch (the library instantiates
// K = 3): the two-step march with more collision stages, so the populations
// cross HBM once per K updates.
// With H = 2K - 1 halo rows, per march position j:
//   stage 0: pull f(t) of row j + H (loads issued PF rows ahead), publish
//            psi(t) into psi ring 0;
//   stage k = 1 .. K-1: collide row j + H - 2k + 1 with psi ring k - 1 into
//            f* ring k; pull f(t + k) of row j + H - 2k from that ring and
//            publish psi(t + k) into psi ring k;
//   last:    collide row j with psi ring K - 1 and store it.
// 2K - 1 barriers per row; H halo rows above and below a band and H halo
// columns on each side of a strip (W <= NT - 2H).  Stage k's collision
// covers ring columns [2k - 1, NT - 2k], its pull [2k, NT - 1 - 2k].  FP32
// values go through the rings unrounded, so a launch is bitwise K single
// steps.
template <int NT, int PF, int W, int K>
__device__ __forceinline__ void multi_step_march(const InstDesc* __restrict__ descs,
                                                 const TileItem* __restrict__ items,
                                                 const int* __restrict__ nitems_p, int sub) {
  static_assert(K == 3 || K == 4, "three or four steps per launch");
  static_assert(PF == 1 || PF == 2, "one or two rows of loads in flight");
  constexpr int H = 2 * K - 1;
  using S = StoreF32;
  using F = Fused2<S, NT, PF, W, H>;
  // FP32 rows are loaded straight into the registers they are collided in:
  // a slot lives from its loads to the first collision, PF + 2 positions.
  constexpr int NR = PF + 2;
  // a multiple of NR, 2 and 3: every slot and ring index is a constant
  constexpr int U = NR == 3 ? 6 : 12;
  static_assert(U % NR == 0 && U % 6 == 0, "unroll period");
  // psi ring k holds psi(t + k) of three consecutive rows
  __shared__ float ps[K][3][NT];
  // f* ring k (k = 1 .. K-1, index k - 1): populations 0, 1, 3 of the
  // middle row (two rows), the side populations of the row collided at this
  // position (one row) and those of the rows collided up to two positions
  // earlier (three rows); which side is which follows the march direction
  __shared__ float rmd[K - 1][2][3][NT], rnew[K - 1][3][NT], rold[K - 1][3][3][NT];
  const int nitems = *nitems_p;
  const int t = strip_slot<S, NT, H>();
  const int strip_f = min(max(t, 1), NT - 2);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const TileItem ti = items[__builtin_amdgcn_readfirstlane(it)];
    const InstDesc* __restrict__ dp = descs + __builtin_amdgcn_readfirstlane(ti.inst);
    if (multi_runs(dp, sub, K)) {
      F s;
      s.setup(dp, ti, sub);
      const int h = s.h;
      uint64_t bad = 0;
      auto march = [&](auto upward, auto wrap_c) {
        const int below = upward ? 1 : -1;
        constexpr bool kW = decltype(wrap_c)::value;
        const int nx = s.nx;
        // lanes of stage k's collision and pull (a periodic strip: every
        // column of the grid)
        bool col_ok[K], pull_ok[K];
#pragma unroll
        for (int k = 1; k < K; ++k) {
          col_ok[k] = kW ? t < nx : (t >= 2 * k - 1 && t <= NT - 2 * k);
          pull_ok[k] = kW ? t < nx : (t >= 2 * k && t <= NT - 1 - 2 * k);
        }
        const int tl = kW ? (t == 0 ? nx - 1 : t - 1) : t - 1;
        const int tr = kW ? (t == nx - 1 ? 0 : min(t + 1, NT - 1)) : t + 1;
        const int tf = kW ? t : strip_f;
        const int tfl = kW ? tl : tf - 1, tfr = kW ? tr : tf + 1;
        float fa[NR][10], fr[K - 1][2][10];
        // Row R (>= -H) of the first step is loaded into slot R mod NR.
        auto fetch_row = [&](int row, auto slot_c) {
          s.fetch(row, fa[decltype(slot_c)::value], nullptr);
        };
        unrolled(std::make_integer_sequence<int, PF>{}, [&](auto k) {
          fetch_row(-H + decltype(k)::value,
                    std::integral_constant<int, (decltype(k)::value + H * NR - H) % NR>{});
        });
        auto pos = [&](auto lead_c, auto u_c, int j) {
          constexpr bool kLead = decltype(lead_c)::value;
          constexpr int u = decltype(u_c)::value;
          // ring slots of row j + d: three-row rings (d >= -9), two-row rings
          auto ring = [&](int d) { return (u + d + 9) % 3; };
          auto ring2 = [&](int d) { return (u + d + 10) % 2; };
          float(&fa_c)[10] = fa[(u + H) % NR];
          fetch_row(min(j + H + PF, h + H - 1),
                    std::integral_constant<int, (u + H + PF) % NR>{});
          fa_c[9] = density(fa_c);
          ps[0][ring(H)][t] = psi_of(fa_c[9]);
          __syncthreads();
          unrolled(std::make_integer_sequence<int, K - 1>{}, [&](auto kc) {
            constexpr int k = decltype(kc)::value + 1;
            constexpr int rc = H - 2 * k + 1;  // row collided at this stage
            constexpr int rp = H - 2 * k;      // row pulled at this stage
            float(&fp)[10] = k == 1 ? fa[(u + rc) % NR] : fr[k >= 2 ? k - 2 : 0][u & 1];
            if ((!kLead || j >= -2 * H + 4 * k - 2) && col_ok[k]) {
              float Fx, Fy;
              ring_force(ps[k - 1][ring(rc + below)], ps[k - 1][ring(rc)],
                         ps[k - 1][ring(rc - below)], t, tl, tr, s.G, Fx, Fy);
              collide(fp, fp[9], Fx, Fy, s.tau, s.omega);
              float(*md)[NT] = rmd[k - 1][ring2(rc)];
              float(*old)[NT] = rold[k - 1][ring(rc)];
              float(*dn)[NT] = upward ? rnew[k - 1] : old;
              float(*up)[NT] = upward ? old : rnew[k - 1];
              md[0][t] = fp[0];
              md[1][t] = fp[1];
              md[2][t] = fp[3];
              dn[0][t] = fp[2];
              dn[1][t] = fp[5];
              dn[2][t] = fp[6];
              up[0][t] = fp[4];
              up[1][t] = fp[7];
              up[2][t] = fp[8];
            }
            __syncthreads();
            if ((!kLead || j >= -2 * H + 4 * k) && pull_ok[k]) {
              // f_i(x) = f*_i(x - e_i): the middle row's rest and horizontal
              // populations, the vertical ones from the rows collided at this
              // position and one position earlier
              float(&f)[10] = fr[k - 1][(u + 1) & 1];
              const float(*md)[NT] = rmd[k - 1][ring2(rp)];
              const float(*old)[NT] = rold[k - 1][ring(rp - 1)];
              const float(*dn)[NT] = upward ? rnew[k - 1] : old;
              const float(*up)[NT] = upward ? old : rnew[k - 1];
              f[0] = md[0][t];
              f[1] = md[1][tl];
              f[2] = dn[0][t];
              f[3] = md[2][tr];
              f[4] = up[0][t];
              f[5] = dn[1][tl];
              f[6] = dn[2][tr];
              f[7] = up[1][tr];
              f[8] = up[2][tl];
              f[9] = density(f);
              ps[k][ring(rp)][t] = psi_of(f[9]);
            }
            __syncthreads();
          });
          if constexpr (!kLead) {
            float(&fp)[10] = fr[K - 2][u & 1];
            float Fx, Fy;
            ring_force(ps[K - 1][ring(below)], ps[K - 1][ring(0)], ps[K - 1][ring(-below)], tf,
                       tfl, tfr, s.G, Fx, Fy);
            bad |= unstable_lanes(fp[9], s.out);
            collide(fp, fp[9], Fx, Fy, s.tau, s.omega);
            s.store(j, fp);
          }
        };
        // 2H lead-in positions, j = -2H .. -1
        unrolled(std::make_integer_sequence<int, 2 * H>{}, [&](auto k) {
          constexpr int j = decltype(k)::value - 2 * H;
          pos(std::true_type{}, std::integral_constant<int, (j % U + U) % U>{}, j);
        });
        const auto phases = std::make_integer_sequence<int, U>{};
        int j0 = 0;
        for (; j0 + U <= h; j0 += U)
          unrolled(phases, [&](auto u) { pos(std::false_type{}, u, j0 + decltype(u)::value); });
        unrolled(std::make_integer_sequence<int, U - 1>{}, [&](auto u) {
          if (j0 + decltype(u)::value < h) pos(std::false_type{}, u, j0 + decltype(u)::value);
        });
      };
      auto go = [&](auto wrap_c) {
        if (s.dir)
          march(std::true_type{}, wrap_c);
        else
          march(std::false_type{}, wrap_c);
      };
      if (s.wrap)
        go(std::true_type{});
      else
        go(std::false_type{});
      report_unstable(dp, bad);
    }
    __syncthreads();  // the next item reuses the rings
  }
}

template <int NT, int PF, int W>
__global__ __launch_bounds__(NT) void k_step3(const InstDesc* __restrict__ descs,
                                              const TileItem* __restrict__ items,
                                              const int* __restrict__ nitems_p, int sub) {
  multi_step_march<NT, PF, W, 3>(descs, items, nitems_p, sub);
}

// Two steps that also record the diagnostics of the state they advance (one
// partial record of kPartialStride doubles per item, folded afterwards).
constexpr int kDiag2Threads = 256;
template <class S>
__global__ __launch_bounds__(kDiag2Threads) void k_step2_diag(const InstDesc* __restrict__ descs,
                                                              const TileItem* __restrict__ items,
                                                              const int* __restrict__ nitems_p,
                                                              int sub,
                                                              double* __restrict__ partials) {
  static_assert(kDiag2Threads == kSeriesThreads, "the recording tile's workgroup");
  constexpr int W = std::is_same<S, StoreF32>::value ? kSeries2WidthF32 : kDiag2Threads - kFusedHalo;
  two_step_march<S, kDiag2Threads, 1, W, true>(descs, items, nitems_p, sub, partials);
}

// ============================================================== batched ticks

// Start of a graph replay: every simulation takes min(K, remaining) steps.
__global__ void k_tick_begin(InstDesc* descs, int n, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int64_t rem = descs[i].remaining;
    descs[i].nsub = (int32_t)(rem < K ? (rem > 0 ? rem : 0) : K);
  }
}

// Before a run of replays: every simulation of the batch has `steps` to take.
__global__ void k_batch_arm(InstDesc* descs, int n, int64_t steps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    descs[i].remaining = steps;
    descs[i].nsub = 0;
  }
}

// End of a graph replay: account for the steps taken (one buffer swap per
// launch that ran).
__global__ void k_tick_end(InstDesc* descs, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int32_t s = descs[i].nsub;
    descs[i].parity = (int32_t)((descs[i].parity + tick_flips(s, launch_steps(descs + i))) & 1);
    descs[i].remaining -= s;
    descs[i].steps += s;
    descs[i].nsub = 0;
  }
}

// ============================================================== cell-parallel helpers

// The nine values a cell stores, A_i(x) for i = 0..8: packed with the global
// shift, or (per-cell-shift storage) with the cell's own reference density
// half(sum_i A_i), which is stored beside them.
template <class S>
__device__ __forceinline__ void store_cell(typename S::T* dst, int nx, int ny, int x, int y,
                                           const float (&a)[9], float rho0) {
  const float ws[9] = {kW0, kW1, kW1, kW1, kW1, kW2, kW2, kW2, kW2};
  if constexpr (S::kMoment) {
    // the record of values whose mass is their sum in index order
    const float r = density(a);
    float jx, jy;
    _Float16 h[6];
    mom_encode(a, r, jx, jy, h);
    char* b = reinterpret_cast<char*>(dst) + mom_row(y, nx);
    *reinterpret_cast<float*>(b + mom_f32(0, nx) + 4ull * x) = r;
    *reinterpret_cast<float*>(b + mom_f32(1, nx) + 4ull * x) = jx;
    *reinterpret_cast<float*>(b + mom_f32(2, nx) + 4ull * x) = jy;
#pragma unroll
    for (int i = 3; i < 9; ++i)
      *reinterpret_cast<_Float16*>(b + mom_f16(i, nx) + 2ull * x) = h[i - 3];
  } else if constexpr (S::kCellShift) {
    float r = a[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) r += a[i];
    const typename S::T rh = S::ref(r);
#pragma unroll
    for (int i = 0; i < 9; ++i) dst[pop_index(i, x, y, nx, ny)] = S::encode(a[i], rh, ws[i]);
    dst[rhat_row(y, nx, ny) + (uint64_t)x] = rh;
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) dst[pop_index(i, x, y, nx, ny)] = S::pack(a[i], ws[i] * rho0);
  }
}

// Moments, pass 1: rho (FP32, the step kernel's summation order).
template <class S>
__global__ __launch_bounds__(256) void k_rho32(const typename S::T* __restrict__ src, int nx,
                                               int ny, float rho0, float* __restrict__ rho) {
  const size_t n = (size_t)nx * ny;
  for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    float f[9];
    pull_cell<S>(src, n, nx, ny, (int)(c % nx), (int)(c / nx), rho0, f);
    rho[c] = density(f);
  }
}

// Moments, pass 2: u = (j + F / 2) / rho with the step kernel's force.
template <class S>
__global__ __launch_bounds__(256) void k_velocity(const typename S::T* __restrict__ src, int nx,
                                                  int ny, float rho0, float G,
                                                  const float* __restrict__ rho,
                                                  float* __restrict__ ux, float* __restrict__ uy) {
  const size_t n = (size_t)nx * ny;
  for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % nx), y = (int)(c / nx);
    const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
    const size_t r0 = (size_t)y * nx, rm = (size_t)wrap_dec(y, ny) * nx,
                 rp = (size_t)wrap_inc(y, ny) * nx;
    float Fx, Fy;
    force_of(psi_of(rho[r0 + x]), psi_of(rho[r0 + xp]), psi_of(rho[rp + x]), psi_of(rho[r0 + xm]),
             psi_of(rho[rm + x]), psi_of(rho[rp + xp]), psi_of(rho[rp + xm]),
             psi_of(rho[rm + xm]), psi_of(rho[rm + xp]), G, Fx, Fy);
    float f[9];
    pull_cell<S>(src, n, nx, ny, x, y, rho0, f);
    float jx, jy;
    momentum(f, jx, jy);
    const float r = rho[c];
    if (ux) ux[c] = fmaf(0.5f, Fx, jx) / r;
    if (uy) uy[c] = fmaf(0.5f, Fy, jy) / r;
  }
}

// State export: pulled pre-collision populations as FP32 planes.
template <class S>
__global__ __launch_bounds__(256) void k_get_state(const typename S::T* __restrict__ src, int nx,
                                                   int ny, float rho0, float* __restrict__ f_out) {
  const size_t n = (size_t)nx * ny;
  for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    float f[9];
    pull_cell<S>(src, n, nx, ny, (int)(c % nx), (int)(c / nx), rho0, f);
#pragma unroll
    for (int i = 0; i < 9; ++i) f_out[i * n + c] = f[i];
  }
}

// State import: A_i(x) = f_i(x + e_i), so that the next pull returns f.
template <class S>
__global__ __launch_bounds__(256) void k_set_state(const float* __restrict__ f_in, int nx, int ny,
                                                   float rho0, typename S::T* __restrict__ dst) {
  const size_t n = (size_t)nx * ny;
  const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % nx), y = (int)(c / nx);
    float a[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int xs = x + ex[i], ys = y + ey[i];
      xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
      ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
      a[i] = f_in[i * n + (size_t)ys * nx + xs];
    }
    store_cell<S>(dst, nx, ny, x, y, a, rho0);
  }
}

// ============================================================== initial droplet

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator: the
// k-th output of the stream seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// rho(x) = rho_g + (rho_l - rho_g) max_k s_k(x) + eta(x) in FP64 (see lbm_init).
// A workgroup covers a 16 x 16 tile of cells.  Droplets are staged through
// LDS in chunks of 256, keeping only those that can reach the tile: once
// (r - R) / width >= 20 the factor 1 - tanh rounds to exactly zero in FP64,
// so a droplet farther than R + 20 width from every cell of the tile (tested
// against the tile centre and its half-diagonal) leaves max_k s_k unchanged.
// The maximum does not depend on the order the kept droplets are visited in.
constexpr int kInitTile = 16;

__global__ __launch_bounds__(256) void k_init_rho(const double* __restrict__ drops, int nd,
                                                  InitArgs a, double* __restrict__ rho) {
  __shared__ double sd[256 * 3];
  __shared__ int near_n;
  const int tx = threadIdx.x % kInitTile, ty = threadIdx.x / kInitTile;
  const int ntx = (a.nx + kInitTile - 1) / kInitTile, nty = (a.ny + kInitTile - 1) / kInitTile;
  const double px = (double)a.period_x, py = (double)a.period_y;
  const double reach = 0.5 * (kInitTile - 1) * 1.4142135623730951 + 1.0;
  for (int t = blockIdx.x; t < ntx * nty; t += gridDim.x) {
    const int bx = (t % ntx) * kInitTile, by = (t / ntx) * kInitTile;
    const int x = bx + tx, y = by + ty;
    const bool ok = x < a.nx && y < a.ny;
    const int64_t gx = a.origin_x + x, gy = a.origin_y + y;
    const double tcx = (double)(a.origin_x + bx) + 0.5 * (kInitTile - 1);
    const double tcy = (double)(a.origin_y + by) + 0.5 * (kInitTile - 1);
    double smax = 0.0;
    for (int k0 = 0; k0 < nd; k0 += 256) {
      const int cnt = min(256, nd - k0);
      __syncthreads();
      if (threadIdx.x == 0) near_n = 0;
      __syncthreads();
      if ((int)threadIdx.x < cnt) {
        const double cx = drops[(size_t)(k0 + threadIdx.x) * 3 + 0];
        const double cy = drops[(size_t)(k0 + threadIdx.x) * 3 + 1];
        const double R = drops[(size_t)(k0 + threadIdx.x) * 3 + 2];
        double dx = tcx - cx, dy = tcy - cy;
        dx -= px * floor(dx / px + 0.5);
        dy -= py * floor(dy / py + 0.5);
        if (sqrt(dx * dx + dy * dy) - reach < R + 20.0 * a.width) {
          const int q = atomicAdd(&near_n, 1);
          sd[3 * q + 0] = cx;
          sd[3 * q + 1] = cy;
          sd[3 * q + 2] = R;
        }
      }
      __syncthreads();
      const int nn = near_n;
      for (int k = 0; k < nn; ++k) {
        double dx = (double)gx - sd[3 * k + 0];
        double dy = (double)gy - sd[3 * k + 1];
        dx -= px * floor(dx / px + 0.5);
        dy -= py * floor(dy / py + 0.5);
        const double r = sqrt(dx * dx + dy * dy);
        const double arg = (r - sd[3 * k + 2]) / a.width;
        if (arg < 20.0) {
          const double s = 0.5 * (1.0 - tanh(arg));
          if (s > smax) smax = s;
        }
      }
    }
    if (ok) {
      const uint64_t gidx = (uint64_t)gy * (uint64_t)a.period_x + (uint64_t)gx;
      const double u = (double)(splitmix64_at(a.seed, gidx) >> 11) * (1.0 / 9007199254740992.0);
      const double eta = a.noise_amp * (2.0 * u - 1.0);
      rho[(size_t)y * a.nx + x] = a.rho_g + (a.rho_l - a.rho_g) * smax + eta;
    }
  }
}

// Fluid at rest, written pull-shifted: A_i(x) = w_i rho(x + e_i).
template <class S>
__global__ __launch_bounds__(256) void k_init_pop(const double* __restrict__ rho, int nx, int ny,
                                                  float rho0, typename S::T* __restrict__ dst) {
  const size_t n = (size_t)nx * ny;
  const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double wd[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                        1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % nx), y = (int)(c / nx);
    float a[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int xs = x + ex[i], ys = y + ey[i];
      xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
      ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
      a[i] = (float)(wd[i] * rho[(size_t)ys * nx + xs]);
    }
    store_cell<S>(dst, nx, ny, x, y, a, rho0);
  }
}

// ============================================================== FP64 reductions

constexpr int kRedThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide reduction of NV values with per-value operator (0 sum, 1 max,
// 2 min), in a fixed order; thread 0 gets the results in v.
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const int (&op)[NV]) {
  __shared__ double part[kRedThreads / 64][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    v[q] = op[q] == 0 ? wave_sum(v[q]) : (op[q] == 1 ? wave_max(v[q]) : wave_min(v[q]));
    if (lane == 0) part[wid][q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double a = part[0][q];
      for (int w = 1; w < kRedThreads / 64; ++w)
        a = op[q] == 0 ? a + part[w][q] : (op[q] == 1 ? fmax(a, part[w][q]) : fmin(a, part[w][q]));
      v[q] = a;
    }
  }
  __syncthreads();
}

// Diagnostics pass 1: rho in FP64 (sum of the widened populations in index
// order) into a scratch plane, plus mass, momentum and a count of cells that
// are not finite or have rho <= 0.  Partials per block: [0..3].
template <class S>
__global__ __launch_bounds__(kRedThreads) void k_diag_rho(const typename S::T* __restrict__ src,
                                                          int nx, int ny, float rho0,
                                                          double* __restrict__ rho64,
                                                          double* __restrict__ partials) {
  const size_t n = (size_t)nx * ny;
  double m = 0.0, px = 0.0, py = 0.0, bad = 0.0;
  for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    float f[9];
    pull_cell<S>(src, n, nx, ny, (int)(c % nx), (int)(c / nx), rho0, f);
    double r = 0.0;
    bool fin = true;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      r += (double)f[i];
      fin = fin && isfinite(f[i]);
    }
    const double jx = ((double)f[1] - (double)f[3]) + ((double)f[5] - (double)f[6]) +
                      ((double)f[8] - (double)f[7]);
    const double jy = ((double)f[2] - (double)f[4]) + ((double)f[5] - (double)f[8]) +
                      ((double)f[6] - (double)f[7]);
    rho64[c] = r;
    m += r;
    px += jx;
    py += jy;
    if (!fin || !(r > 0.0)) bad += 1.0;
  }
  double v[4] = {m, px, py, bad};
  const int op[4] = {0, 0, 0, 0};
  block_reduce<4>(v, op);
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) partials[blockIdx.x * kPartialStride + q] = v[q];
}

// Diagnostics pass 2: Eq. (16) |grad rho| with periodic wrap, and the sums
// and extrema of Eqs. (9)-(15).  Partials per block: [4..9].
__global__ __launch_bounds__(kRedThreads) void k_diag_grad(const double* __restrict__ rho, int nx,
                                                           int ny, double* __restrict__ partials) {
  const size_t n = (size_t)nx * ny;
  double cnt = 0.0, gmax = 0.0, gsum = 0.0, g2 = 0.0, rmax = -INFINITY, rmin = INFINITY;
  for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n;
       c += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % nx), y = (int)(c / nx);
    const size_t r0 = (size_t)y * nx;
    const double gx = (rho[r0 + wrap_inc(x, nx)] - rho[r0 + wrap_dec(x, nx)]) / 2.0;
    const double gy = (rho[(size_t)wrap_inc(y, ny) * nx + x] - rho[(size_t)wrap_dec(y, ny) * nx + x]) / 2.0;
    const double g = sqrt(gx * gx + gy * gy);
    const double r = rho[c];
    if (g > 0.01) cnt += 1.0;
    gmax = fmax(gmax, g);
    gsum += g;
    g2 += g * g;
    rmax = fmax(rmax, r);
    rmin = fmin(rmin, r);
  }
  double v[6] = {cnt, gmax, gsum, g2, rmax, rmin};
  const int op[6] = {0, 1, 0, 0, 1, 2};
  block_reduce<6>(v, op);
  if (threadIdx.x == 0)
    for (int q = 0; q < 6; ++q) partials[blockIdx.x * kPartialStride + 4 + q] = v[q];
}

// Final pass: one block folds the per-block partials in a fixed order.
__global__ __launch_bounds__(kRedThreads) void k_diag_final(const double* __restrict__ partials,
                                                            int nblocks, double* __restrict__ out) {
  const int op10[10] = {0, 0, 0, 0, 0, 1, 0, 0, 1, 2};
  double v[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) v[q] = op10[q] == 1 ? -INFINITY : (op10[q] == 2 ? INFINITY : 0.0);
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const double p = partials[b * kPartialStride + q];
      v[q] = op10[q] == 0 ? v[q] + p : (op10[q] == 1 ? fmax(v[q], p) : fmin(v[q], p));
    }
  }
  block_reduce<10>(v, op10);
  if (threadIdx.x == 0)
    for (int q = 0; q < 10; ++q) out[q] = v[q];
}

// ============================================================== bandwidth reference

// Streaming copy, one 16-byte vector per thread and pass.  On gfx950 this is
// the fastest of the forms timed over 2 GiB (6.1 TB/s; four vectors per
// thread in a grid-stride loop reached 4.5 TB/s, eight per thread 5.4).
__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src,
                                              float4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

// ============================================================== launchers

namespace {

template <class S, int NT, int CPT, int PF>
hipError_t launch_step_t(const InstDesc* descs, const TileItem* items, const int* nitems,
                         int grid, int sub, hipStream_t st) {
  hipLaunchKernelGGL((k_step<S, NT, CPT, PF>), dim3(grid), dim3(NT), 0, st, descs, items, nitems,
                     sub);
  return hipGetLastError();
}

template <class S, int NT, int CPT, int PF>
const void* step_fn_t() {
  return reinterpret_cast<const void*>(&k_step<S, NT, CPT, PF>);
}

// Moment storage has no paired-column kernel, and two-step kernels only for
// strips of at most NT - 8 columns (four halo columns on each side); the
// other shapes are not valid tiles for it (tile_valid).
template <class S, int NT, int PF, int W>
hipError_t launch_fused_t(const InstDesc* descs, const TileItem* items, const int* nitems,
                          int grid, int sub, hipStream_t st) {
  if constexpr (W > NT - 2 * fused_halo<S>()) {
    return hipErrorInvalidDeviceFunction;
  } else {
    hipLaunchKernelGGL((k_step2<S, NT, PF, W>), dim3(grid), dim3(NT), 0, st, descs, items, nitems,
                       sub);
    return hipGetLastError();
  }
}

template <class S, int NT, int PF, int W>
const void* fused_fn_t() {
  if constexpr (W > NT - 2 * fused_halo<S>())
    return nullptr;
  else
    return reinterpret_cast<const void*>(&k_step2<S, NT, PF, W>);
}

// Kernels of more than two steps per launch: FP32 storage only.
template <int K, int NT, int PF, int W>
constexpr auto multi_kernel() {
  static_assert(K == 3, "three steps per launch");
  return &k_step3<NT, PF, W>;
}

template <class S, int K, int NT, int PF, int W>
hipError_t launch_multi_t(const InstDesc* descs, const TileItem* items, const int* nitems,
                          int grid, int sub, hipStream_t st) {
  if constexpr (!std::is_same<S, StoreF32>::value) {
    return hipErrorInvalidDeviceFunction;
  } else {
    constexpr auto kern = multi_kernel<K, NT, PF, W>();
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, st, descs, items, nitems, sub);
    return hipGetLastError();
  }
}

template <class S, int K, int NT, int PF, int W>
const void* multi_fn_t() {
  if constexpr (!std::is_same<S, StoreF32>::value)
    return nullptr;
  else
    return reinterpret_cast<const void*>(multi_kernel<K, NT, PF, W>());
}

template <class S, int NW, int PF>
hipError_t launch_pair_t(const InstDesc* descs, const TileItem* items, const int* nitems,
                         int grid, int sub, hipStream_t st) {
  if constexpr (S::kMoment) {
    return hipErrorInvalidDeviceFunction;
  } else {
    hipLaunchKernelGGL((k_step_pair<S, NW, PF>), dim3(grid), dim3(64 * NW), 0, st, descs, items,
                       nitems, sub);
    return hipGetLastError();
  }
}

template <class S, int NW, int PF>
const void* pair_fn_t() {
  if constexpr (S::kMoment)
    return nullptr;
  else
    return reinterpret_cast<const void*>(&k_step_pair<S, NW, PF>);
}

using StepLauncher = hipError_t (*)(const InstDesc*, const TileItem*, const int*, int, int,
                                    hipStream_t);
using StepFn = const void* (*)();

// Step-kernel variants (threads, cells per thread, rows in flight); the order
// fixes the tile-shape numbering.
#define SCLBM_STEP_VARIANTS(X)                                                          \
  X(64, 1, 1) X(64, 1, 2) X(128, 1, 1) X(128, 1, 2) X(64, 4, 1) X(128, 2, 1) X(128, 2, 2) \
  X(256, 1, 1) X(256, 1, 2) X(256, 2, 1) X(512, 1, 1) X(512, 1, 2) X(256, 2, 2)         \
  X(1024, 1, 1)

// Paired-column variants (wavefronts per workgroup, rows in flight).
#define SCLBM_PAIR_VARIANTS(X) X(1, 1) X(1, 2) X(2, 1) X(2, 2) X(4, 1) X(4, 2)

// Two-step variants (threads, rows in flight).
// Two-step variants (threads, rows in flight, output columns): the widest
// strips, and strips of a multiple of 16 columns (64-byte aligned in FP32).
#define SCLBM_FUSED_VARIANTS(X)                                                               \
  X(128, 1, 122) X(256, 1, 250) X(256, 2, 250) X(512, 1, 506) X(512, 2, 506) X(128, 1, 112) \
  X(256, 1, 240) X(256, 2, 240) X(512, 1, 496)

// Three-step variants (FP32): strips of a multiple of 16 columns with five
// halo columns on each side.
#define SCLBM_MULTI_VARIANTS(X) X(3, 128, 1, 112) X(3, 256, 1, 240) X(3, 256, 2, 240) X(3, 512, 1, 496)

#define SCLBM_AS_VARIANT(NT, CPT, PF) StepVariant{NT, CPT, PF, 0, 1, 0},
#define SCLBM_AS_LAUNCH(NT, CPT, PF) launch_step_t<S, NT, CPT, PF>,
#define SCLBM_AS_FN(NT, CPT, PF) step_fn_t<S, NT, CPT, PF>,
#define SCLBM_PAIR_AS_VARIANT(NW, PF) StepVariant{64 * NW, 2, PF, 1, 1, 0},
#define SCLBM_PAIR_AS_LAUNCH(NW, PF) launch_pair_t<S, NW, PF>,
#define SCLBM_PAIR_AS_FN(NW, PF) pair_fn_t<S, NW, PF>,
#define SCLBM_FUSED_AS_VARIANT(NT, PF, W) StepVariant{NT, 1, PF, 0, 2, W},
#define SCLBM_FUSED_AS_LAUNCH(NT, PF, W) launch_fused_t<S, NT, PF, W>,
#define SCLBM_FUSED_AS_FN(NT, PF, W) fused_fn_t<S, NT, PF, W>,
#define SCLBM_MULTI_AS_VARIANT(K, NT, PF, W) StepVariant{NT, 1, PF, 0, K, W},
#define SCLBM_MULTI_AS_LAUNCH(K, NT, PF, W) launch_multi_t<S, K, NT, PF, W>,
#define SCLBM_MULTI_AS_FN(K, NT, PF, W) multi_fn_t<S, K, NT, PF, W>,
constexpr StepVariant kVariants[] = {
    SCLBM_STEP_VARIANTS(SCLBM_AS_VARIANT) SCLBM_PAIR_VARIANTS(SCLBM_PAIR_AS_VARIANT)
        SCLBM_FUSED_VARIANTS(SCLBM_FUSED_AS_VARIANT) SCLBM_MULTI_VARIANTS(SCLBM_MULTI_AS_VARIANT)};
template <class S>
constexpr StepLauncher kLaunch[] = {
    SCLBM_STEP_VARIANTS(SCLBM_AS_LAUNCH) SCLBM_PAIR_VARIANTS(SCLBM_PAIR_AS_LAUNCH)
        SCLBM_FUSED_VARIANTS(SCLBM_FUSED_AS_LAUNCH) SCLBM_MULTI_VARIANTS(SCLBM_MULTI_AS_LAUNCH)};
template <class S>
constexpr StepFn kFn[] = {SCLBM_STEP_VARIANTS(SCLBM_AS_FN) SCLBM_PAIR_VARIANTS(SCLBM_PAIR_AS_FN)
                              SCLBM_FUSED_VARIANTS(SCLBM_FUSED_AS_FN)
                                  SCLBM_MULTI_VARIANTS(SCLBM_MULTI_AS_FN)};
#undef SCLBM_AS_VARIANT
#undef SCLBM_AS_LAUNCH
#undef SCLBM_AS_FN
#undef SCLBM_PAIR_AS_VARIANT
#undef SCLBM_PAIR_AS_LAUNCH
#undef SCLBM_PAIR_AS_FN
#undef SCLBM_FUSED_AS_VARIANT
#undef SCLBM_FUSED_AS_LAUNCH
#undef SCLBM_FUSED_AS_FN
#undef SCLBM_MULTI_AS_VARIANT
#undef SCLBM_MULTI_AS_LAUNCH
#undef SCLBM_MULTI_AS_FN

static_assert(sizeof(kVariants) / sizeof(kVariants[0]) == kNumVariants, "variant table");

int grid_for(size_t n, int threads, int cap) {
  size_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > (size_t)cap) g = cap;
  return (int)g;
}

}  // namespace

const StepVariant& step_variant(int v) { return kVariants[v]; }

namespace {
const void* step_fn(int storage, int variant) {
  switch (storage) {
    case 0: return kFn<StoreF32>[variant]();
    case 1: return kFn<StoreF16S>[variant]();
    case 2: return kFn<StoreF16C>[variant]();
    default: return kFn<StoreF16M>[variant]();
  }
}
}  // namespace

hipError_t launch_step(int storage, int variant, const InstDesc* descs, const TileItem* items,
                       const int* nitems, int grid, int sub, hipStream_t st) {
  switch (storage) {
    case 0: return kLaunch<StoreF32>[variant](descs, items, nitems, grid, sub, st);
    case 1: return kLaunch<StoreF16S>[variant](descs, items, nitems, grid, sub, st);
    case 2: return kLaunch<StoreF16C>[variant](descs, items, nitems, grid, sub, st);
    default: return kLaunch<StoreF16M>[variant](descs, items, nitems, grid, sub, st);
  }
}

hipError_t step_occupancy(int storage, int variant, int* blocks_per_cu) {
  const void* fn = step_fn(storage, variant);
  if (!fn) return hipErrorInvalidDeviceFunction;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn,
                                                      kVariants[variant].threads, 0);
}

hipError_t launch_tick_end(InstDesc* descs, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_tick_end, dim3((n + 255) / 256), dim3(256), 0, st, descs, n);
  return hipGetLastError();
}

hipError_t launch_batch_arm(InstDesc* descs, int n, int64_t steps, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_arm, dim3((n + 255) / 256), dim3(256), 0, st, descs, n, steps);
  return hipGetLastError();
}

hipError_t graph_add_step(hipGraph_t g, hipGraphNode_t* node, const hipGraphNode_t* deps, size_t nd,
                          int storage, int variant, const InstDesc* descs, const TileItem* items,
                          const int* nitems, int grid, int sub) {
  void* args[] = {(void*)&descs, (void*)&items, (void*)&nitems, (void*)&sub};
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(step_fn(storage, variant));
  kp.gridDim = dim3(grid);
  kp.blockDim = dim3(kVariants[variant].threads);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  return hipGraphAddKernelNode(node, g, deps, nd, &kp);
}

hipError_t graph_add_tick(hipGraph_t g, hipGraphNode_t* node, const hipGraphNode_t* deps,
                          size_t nd, bool begin, InstDesc* descs, int n, int K) {
  hipKernelNodeParams kp{};
  void* args_b[] = {(void*)&descs, (void*)&n, (void*)&K};
  void* args_e[] = {(void*)&descs, (void*)&n};
  kp.func = begin ? reinterpret_cast<void*>(&k_tick_begin) : reinterpret_cast<void*>(&k_tick_end);
  kp.gridDim = dim3((n + 255) / 256);
  kp.blockDim = dim3(256);
  kp.sharedMemBytes = 0;
  kp.kernelParams = begin ? args_b : args_e;
  kp.extra = nullptr;
  return hipGraphAddKernelNode(node, g, deps, nd, &kp);
}

// Calls f with a value of the storage trait numbered `storage` (LBM_F32,
// LBM_F16_SHIFTED, LBM_F16_CELL, LBM_F16_MOMENT).
template <class F>
hipError_t with_storage(int storage, F&& f) {
  switch (storage) {
    case 0: return f(StoreF32{});
    case 1: return f(StoreF16S{});
    case 2: return f(StoreF16C{});
    default: return f(StoreF16M{});
  }
}

hipError_t launch_moments(int storage, const void* src, int nx, int ny, float rho0, float G,
                          float* rho, float* ux, float* uy, hipStream_t st) {
  const int g = grid_for((size_t)nx * ny, 256, 8192);
  return with_storage(storage, [&](auto tag) {
    using S = decltype(tag);
    using T = typename S::T;
    hipLaunchKernelGGL(k_rho32<S>, dim3(g), dim3(256), 0, st, (const T*)src, nx, ny, rho0, rho);
    if (ux || uy)
      hipLaunchKernelGGL(k_velocity<S>, dim3(g), dim3(256), 0, st, (const T*)src, nx, ny, rho0, G,
                         (const float*)rho, ux, uy);
    return hipGetLastError();
  });
}

hipError_t launch_get_state(int storage, const void* src, int nx, int ny, float rho0, float* f,
                            hipStream_t st) {
  const int g = grid_for((size_t)nx * ny, 256, 8192);
  return with_storage(storage, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(k_get_state<S>, dim3(g), dim3(256), 0, st, (const typename S::T*)src, nx,
                       ny, rho0, f);
    return hipGetLastError();
  });
}

hipError_t launch_set_state(int storage, const float* f, int nx, int ny, float rho0, void* dst,
                            hipStream_t st) {
  const int g = grid_for((size_t)nx * ny, 256, 8192);
  return with_storage(storage, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(k_set_state<S>, dim3(g), dim3(256), 0, st, f, nx, ny, rho0,
                       (typename S::T*)dst);
    return hipGetLastError();
  });
}

hipError_t launch_init(int storage, const double* drops, int nd, const InitArgs& a, double* rho64,
                       float rho0, void* dst, hipStream_t st) {
  const size_t n = (size_t)a.nx * a.ny;
  const size_t tiles = (size_t)((a.nx + kInitTile - 1) / kInitTile) * ((a.ny + kInitTile - 1) / kInitTile);
  const int g = (int)std::min<size_t>(tiles, 16384);
  hipLaunchKernelGGL(k_init_rho, dim3(g), dim3(256), 0, st, drops, nd, a, rho64);
  const int g2 = grid_for(n, 256, 8192);
  return with_storage(storage, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(k_init_pop<S>, dim3(g2), dim3(256), 0, st, (const double*)rho64, a.nx, a.ny,
                       rho0, (typename S::T*)dst);
    return hipGetLastError();
  });
}

int diagnostics_blocks(int nx, int ny) {
  return grid_for((size_t)nx * ny, kRedThreads, kMaxPartials);
}

hipError_t launch_diagnostics(int storage, const void* src, int nx, int ny, float rho0,
                              double* rho64, double* partials, double* out, hipStream_t st) {
  const int g = diagnostics_blocks(nx, ny);
  const hipError_t e = with_storage(storage, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(k_diag_rho<S>, dim3(g), dim3(kRedThreads), 0, st, (const typename S::T*)src,
                       nx, ny, rho0, rho64, partials);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_grad, dim3(g), dim3(kRedThreads), 0, st, (const double*)rho64, nx, ny,
                     partials);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kRedThreads), 0, st, (const double*)partials, g,
                     out);
  return hipGetLastError();
}

hipError_t launch_step_diag(int storage, const InstDesc* descs, const TileItem* items,
                            const int* nitems, int grid, int sub, double* partials,
                            double* out, hipStream_t st) {
  const hipError_t e = with_storage(storage, [&](auto tag) {
    using S = decltype(tag);
    hipLaunchKernelGGL(k_step_diag<S>, dim3(grid), dim3(kDiagThreads), 0, st, descs, items, nitems,
                       sub, partials);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kRedThreads), 0, st, (const double*)partials, grid,
                     out);
  return hipGetLastError();
}

hipError_t launch_step2_diag(int storage, const InstDesc* descs, const TileItem* items,
                             const int* nitems, int grid, int sub, double* partials, double* out,
                             hipStream_t st) {
  const hipError_t e = with_storage(storage, [&](auto tag) {
    using S = decltype(tag);
    if constexpr (S::kMoment) {  // moment storage takes single steps only
      return hipErrorInvalidDeviceFunction;
    } else {
      hipLaunchKernelGGL(k_step2_diag<S>, dim3(grid), dim3(kDiag2Threads), 0, st, descs, items,
                         nitems, sub, partials);
      return hipGetLastError();
    }
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kRedThreads), 0, st, (const double*)partials, grid,
                     out);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n, 256, 1 << 22)), dim3(256), 0, st,
                     (const float4*)src, (float4*)dst, n);
  return hipGetLastError();
}

}  // namespace sclbm

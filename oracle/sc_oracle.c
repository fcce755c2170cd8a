/*
 * sc_oracle.c -- plain FP64 CPU oracle of the D2Q9 Shan-Chen pseudopotential
 * lattice Boltzmann time step and of the paper's interface metrics.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only code that loads this file.  The GPU
 * library never links, includes or calls anything here and shares no code,
 * constant table or helper with it.
 *
 * Source: Li & Zhang, "Physics-Informed Neural Networks for Enhanced Interface
 * Preservation in Lattice Boltzmann Multiphase Simulations" (arXiv 2504.10539).
 *   - Sec. II-A, Eq. (1): the evolution equation, collide-with-forcing then
 *     stream along the discrete velocity.
 *   - Sec. II-A: pseudopotential (Shan-Chen) interaction force giving a
 *     non-ideal equation of state.  The paper names the model but not its
 *     lattice, psi, stencil or forcing scheme; this oracle takes the reading
 *     D2Q9, psi = 1 - exp(-rho), F = -G psi(x) sum_i w_i psi(x + e_i) e_i,
 *     BGK collision with the Shan-Chen velocity shift u_eq = u' + tau F / rho.
 *   - Sec. III-A: square domain with periodic boundaries; droplet set-up.
 *   - Sec. II-D, Eqs. (9)-(13) and Sec. IV-E, Eqs. (14)-(16): interface width,
 *     maximum gradient, phase separation, effective width, interface energy,
 *     with the central-difference gradient of Eq. (16).
 *
 * Conventions: lattice units (dx = dt = 1, c_s^2 = 1/3).  Velocities in order
 *   e0 = (0,0); e1..e4 = (1,0) (0,1) (-1,0) (0,-1);
 *   e5..e8 = (1,1) (-1,1) (-1,-1) (1,-1);
 * weights 4/9, 1/9 (axes), 1/36 (diagonals).  Population arrays are
 * f[i][y][x] with x fastest; the state is the pre-collision f(t).
 *
 * Everything is written as the plain definition: no blocking, fusion or
 * reordering.  The per-cell loops may run over OpenMP threads (each cell is
 * computed independently, so the result does not depend on the thread count);
 * the reductions are serial in a fixed order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static long wrapi(long a, long n) {
  long r = a % n;
  return r < 0 ? r + n : r;
}

static size_t at(int nx, int ny, int i, long x, long y) {
  return ((size_t)i * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x;
}

/* Lattice export so that tests can build independent checks in the same
 * population order. */
void oracle_lattice(int* ex, int* ey, double* w) {
  for (int i = 0; i < Q; ++i) {
    ex[i] = EX[i];
    ey[i] = EY[i];
    w[i] = WT[i];
  }
}

/* Pseudopotential psi(rho) = 1 - exp(-rho)  (Sec. II-A, pseudopotential model). */
double oracle_psi(double rho) { return 1.0 - exp(-rho); }

/* Second-order BGK equilibrium
 * f_eq_i = w_i rho [1 + 3 e_i.u + 4.5 (e_i.u)^2 - 1.5 |u|^2]
 * (the collision operator Omega_i of Eq. (1)). */
void oracle_equilibrium(double rho, double ux, double uy, double* feq) {
  double usq = ux * ux + uy * uy;
  for (int i = 0; i < Q; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    feq[i] = WT[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
  }
}

/* rho(x) = sum_i f_i(x). */
void oracle_density(int nx, int ny, const double* f, double* rho) {
  for (long y = 0; y < ny; ++y)
    for (long x = 0; x < nx; ++x) {
      double s = 0.0;
      for (int i = 0; i < Q; ++i) s += f[at(nx, ny, i, x, y)];
      rho[y * nx + x] = s;
    }
}

/* Interaction force from a density field:
 * F(x) = -G psi(x) sum_{i=1..8} w_i psi((x + e_i) mod N) e_i. */
void oracle_force(int nx, int ny, double G, const double* rho, double* Fx,
                  double* Fy) {
  for (long y = 0; y < ny; ++y)
    for (long x = 0; x < nx; ++x) {
      double sx = 0.0, sy = 0.0;
      for (int i = 1; i < Q; ++i) {
        long xn = wrapi(x + EX[i], nx), yn = wrapi(y + EY[i], ny);
        double pn = oracle_psi(rho[yn * nx + xn]);
        sx += WT[i] * pn * EX[i];
        sy += WT[i] * pn * EY[i];
      }
      double p = oracle_psi(rho[y * nx + x]);
      Fx[y * nx + x] = -G * p * sx;
      Fy[y * nx + x] = -G * p * sy;
    }
}

/* One or more time steps of Eq. (1) on the pre-collision state f, in place.
 * Per step:
 *   1. rho = sum_i f_i;  psi = 1 - exp(-rho)
 *   2. F = -G psi(x) sum_i w_i psi(x + e_i) e_i
 *   3. u' = sum_i f_i e_i / rho;  u_eq = u' + tau F / rho   (velocity shift)
 *   4. f*_i = f_i - (f_i - f_eq_i(rho, u_eq)) / tau          (BGK)
 *   5. f_i((x + e_i) mod N, t + 1) = f*_i(x)                   (streaming)
 * Returns 0, or -1 for bad arguments, -2 if memory runs out. */
int oracle_step(int nx, int ny, double G, double tau, double* f, long nsteps,
                int nthreads) {
  if (nx < 1 || ny < 1 || !(tau > 0.0) || nsteps < 0) return -1;
  if (nthreads < 1) nthreads = 1;
  size_t n = (size_t)nx * (size_t)ny;
  double* fn = (double*)malloc(sizeof(double) * Q * n);
  double* psi = (double*)malloc(sizeof(double) * n);
  if (!fn || !psi) {
    free(fn);
    free(psi);
    return -2;
  }
  for (long t = 0; t < nsteps; ++t) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long y = 0; y < ny; ++y)
      for (long x = 0; x < nx; ++x) {
        double rho = 0.0;
        for (int i = 0; i < Q; ++i) rho += f[at(nx, ny, i, x, y)];
        psi[y * nx + x] = oracle_psi(rho);
      }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long y = 0; y < ny; ++y)
      for (long x = 0; x < nx; ++x) {
        double fl[Q], feq[Q];
        double rho = 0.0, jx = 0.0, jy = 0.0;
        for (int i = 0; i < Q; ++i) {
          fl[i] = f[at(nx, ny, i, x, y)];
          rho += fl[i];
          jx += fl[i] * EX[i];
          jy += fl[i] * EY[i];
        }
        double sx = 0.0, sy = 0.0;
        for (int i = 1; i < Q; ++i) {
          long xn = wrapi(x + EX[i], nx), yn = wrapi(y + EY[i], ny);
          double pn = psi[yn * nx + xn];
          sx += WT[i] * pn * EX[i];
          sy += WT[i] * pn * EY[i];
        }
        double p = psi[y * nx + x];
        double Fx = -G * p * sx, Fy = -G * p * sy;
        double ux = jx / rho + tau * Fx / rho;
        double uy = jy / rho + tau * Fy / rho;
        oracle_equilibrium(rho, ux, uy, feq);
        for (int i = 0; i < Q; ++i) {
          double fstar = fl[i] - (fl[i] - feq[i]) / tau;
          long xd = wrapi(x + EX[i], nx), yd = wrapi(y + EY[i], ny);
          fn[at(nx, ny, i, xd, yd)] = fstar;
        }
      }
    memcpy(f, fn, sizeof(double) * Q * n);
  }
  free(fn);
  free(psi);
  return 0;
}

/* Macroscopic fields of the pre-collision state: rho = sum_i f_i and the
 * half-force-corrected velocity u = (sum_i f_i e_i + F / 2) / rho. */
int oracle_moments(int nx, int ny, double G, const double* f, double* rho,
                   double* ux, double* uy) {
  size_t n = (size_t)nx * (size_t)ny;
  double* Fx = (double*)malloc(sizeof(double) * n);
  double* Fy = (double*)malloc(sizeof(double) * n);
  if (!Fx || !Fy) {
    free(Fx);
    free(Fy);
    return -2;
  }
  oracle_density(nx, ny, f, rho);
  oracle_force(nx, ny, G, rho, Fx, Fy);
  for (long y = 0; y < ny; ++y)
    for (long x = 0; x < nx; ++x) {
      double jx = 0.0, jy = 0.0;
      for (int i = 0; i < Q; ++i) {
        jx += f[at(nx, ny, i, x, y)] * EX[i];
        jy += f[at(nx, ny, i, x, y)] * EY[i];
      }
      size_t c = (size_t)y * nx + x;
      ux[c] = (jx + 0.5 * Fx[c]) / rho[c];
      uy[c] = (jy + 0.5 * Fy[c]) / rho[c];
    }
  free(Fx);
  free(Fy);
  return 0;
}

/* Total mass and momentum of the pre-collision state:
 * out = {sum_x sum_i f_i, sum_x sum_i f_i e_ix, sum_x sum_i f_i e_iy}. */
void oracle_conservation(int nx, int ny, const double* f, double* out) {
  double m = 0.0, px = 0.0, py = 0.0;
  for (long y = 0; y < ny; ++y)
    for (long x = 0; x < nx; ++x)
      for (int i = 0; i < Q; ++i) {
        double v = f[at(nx, ny, i, x, y)];
        m += v;
        px += v * EX[i];
        py += v * EY[i];
      }
  out[0] = m;
  out[1] = px;
  out[2] = py;
}

/* Eq. (16): |grad rho|_{i,j} by central differences with dx = dy = 1 and the
 * periodic wrap of the domain (i is the x index, j the y index). */
void oracle_grad_mag(int nx, int ny, const double* rho, double* g) {
  for (long y = 0; y < ny; ++y)
    for (long x = 0; x < nx; ++x) {
      double gx = (rho[y * nx + wrapi(x + 1, nx)] -
                   rho[y * nx + wrapi(x - 1, nx)]) / 2.0;
      double gy = (rho[wrapi(y + 1, ny) * nx + x] -
                   rho[wrapi(y - 1, ny) * nx + x]) / 2.0;
      g[y * nx + x] = sqrt(gx * gx + gy * gy);
    }
}

/* Interface metrics of a density field (Eqs. (9)-(16)), out[]:
 *   0 W      = #cells with |grad rho| > 0.01 / #cells               Eq. (9)
 *   1 G_max  = max |grad rho|                                       Eq. (10)
 *   2 drho   = rho_max - rho_min                                    Eq. (11)
 *   3 W_eff  = sum |grad rho| dx dy / (G_max V_total), 0 if G_max=0 Eqs. (12),(14)
 *   4 E_int  = sum |grad rho|^2 dx dy                               Eqs. (13),(15)
 *   5 count of cells above the threshold, 6 rho_max, 7 rho_min,
 *   8 sum |grad rho|. */
int oracle_metrics(int nx, int ny, const double* rho, double* out) {
  size_t n = (size_t)nx * (size_t)ny;
  double* g = (double*)malloc(sizeof(double) * n);
  if (!g) return -2;
  oracle_grad_mag(nx, ny, rho, g);
  double count = 0.0, gmax = 0.0, gsum = 0.0, g2sum = 0.0;
  double rmax = rho[0], rmin = rho[0];
  for (size_t c = 0; c < n; ++c) {
    if (g[c] > 0.01) count += 1.0;
    if (g[c] > gmax) gmax = g[c];
    gsum += g[c];
    g2sum += g[c] * g[c];
    if (rho[c] > rmax) rmax = rho[c];
    if (rho[c] < rmin) rmin = rho[c];
  }
  double vtotal = (double)n; /* area with dx = dy = 1 */
  out[0] = count / vtotal;
  out[1] = gmax;
  out[2] = rmax - rmin;
  out[3] = gmax > 0.0 ? gsum / (gmax * vtotal) : 0.0;
  out[4] = g2sum;
  out[5] = count;
  out[6] = rmax;
  out[7] = rmin;
  out[8] = gsum;
  free(g);
  return 0;
}

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) used as a counter-based
 * generator: the k-th output (k = 0, 1, ...) of the stream seeded with `seed`. */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Uniform in [0, 1) from the top 53 bits of the k-th output. */
double oracle_uniform01(uint64_t seed, uint64_t k) {
  return (double)(oracle_splitmix64(seed, k) >> 11) * (1.0 / 9007199254740992.0);
}

/* Droplet initial density (Sec. III-A set-up, with the tanh profile, noise and
 * max-merge of overlapping droplets taken as the build's reading):
 *   rho(x) = rho_g + (rho_l - rho_g) max_k s_k(x) + eta(x),
 *   s_k = 0.5 [1 - tanh((r_k - R_k) / width)],
 * r_k the minimum-image distance, in a periodic domain of size
 * period_x x period_y, from the integer cell (origin_x + x, origin_y + y) to
 * the centre (cx_k, cy_k); eta = noise_amp (2u - 1) with u the uniform variate
 * of the global linear index gy * period_x + gx.  The n x 3 array `drops`
 * holds (cx, cy, R).  A period of 0 means the domain itself. */
void oracle_init_density(int nx, int ny, const double* drops, int n,
                         double rho_l, double rho_g, double width,
                         double noise_amp, uint64_t seed, long period_x,
                         long period_y, long origin_x, long origin_y,
                         double* rho) {
  double px = (double)(period_x > 0 ? period_x : nx);
  double py = (double)(period_y > 0 ? period_y : ny);
  long pxl = period_x > 0 ? period_x : nx;
  for (long y = 0; y < ny; ++y)
    for (long x = 0; x < nx; ++x) {
      long gx = origin_x + x, gy = origin_y + y;
      double smax = 0.0;
      for (int k = 0; k < n; ++k) {
        double dx = (double)gx - drops[3 * k + 0];
        double dy = (double)gy - drops[3 * k + 1];
        dx -= px * floor(dx / px + 0.5);
        dy -= py * floor(dy / py + 0.5);
        double r = sqrt(dx * dx + dy * dy);
        double s = 0.5 * (1.0 - tanh((r - drops[3 * k + 2]) / width));
        if (s > smax) smax = s;
      }
      uint64_t gidx = (uint64_t)gy * (uint64_t)pxl + (uint64_t)gx;
      double eta = noise_amp * (2.0 * oracle_uniform01(seed, gidx) - 1.0);
      rho[y * nx + x] = rho_g + (rho_l - rho_g) * smax + eta;
    }
}

/* Fluid at rest: f_i = w_i rho (the equilibrium at u = 0). */
void oracle_init_populations(int nx, int ny, const double* rho, double* f) {
  for (int i = 0; i < Q; ++i)
    for (long y = 0; y < ny; ++y)
      for (long x = 0; x < nx; ++x)
        f[at(nx, ny, i, x, y)] = WT[i] * rho[y * nx + x];
}

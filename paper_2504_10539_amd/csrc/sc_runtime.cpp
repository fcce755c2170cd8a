// sc_runtime.cpp -- host runtime of the D2Q9 Shan-Chen library: single runs,
// tile shapes and their autotuner, batched runs over a HIP graph, and the
// C-ABI entry points declared in include/lbm.h (method: Li & Zhang, arXiv
// 2504.10539, Sec. II-A Eq. (1), Sec. III-A set-up, Eqs. (9)-(16) metrics).
#include "sc_runtime.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace sclbm {

// ------------------------------------------------------------------ errors

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }

lbm_status fail(lbm_status code, const std::string& msg) {
  g_error = msg;
  return code;
}

lbm_status fail_nothrow(lbm_status code, const char* where, const char* what) noexcept {
  try {
    g_error = std::string(where) + ": " + what;
  } catch (...) {
    g_error.clear();
  }
  return code;
}

lbm_status hip_fail(hipError_t e, const char* what) {
  g_error = std::string(what) + ": " + hipGetErrorString(e);
  return LBM_EDEVICE;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

lbm_status validate_params(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nx > 65536 || p->ny > 65536)
    return fail(LBM_EINVAL, "nx and ny must be in [1, 65536]");
  if ((uint64_t)p->nx * (uint64_t)p->ny * 9ull >= (1ull << 32))
    return fail(LBM_EINVAL, "grid too large (9 nx ny must be < 2^32)");
  if (!std::isfinite(p->G)) return fail(LBM_EINVAL, "G must be finite");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_EINVAL, "tau must be > 0.5");
  if (p->storage != LBM_F32 && p->storage != LBM_F16_SHIFTED && p->storage != LBM_F16_CELL &&
      p->storage != LBM_F16_MOMENT)
    return fail(LBM_EINVAL,
                "storage must be LBM_F32, LBM_F16_SHIFTED, LBM_F16_CELL or LBM_F16_MOMENT");
  if (p->storage == LBM_F16_SHIFTED && (!std::isfinite(p->rho0) || p->rho0 < 0.0))
    return fail(LBM_EINVAL, "rho0 must be finite and >= 0");
  return LBM_OK;
}

size_t pop_bytes_for(const lbm_params& p) {
  // moment storage: three FP32 and six FP16 values per cell
  if (p.storage == LBM_F16_MOMENT) return 24ull * (size_t)p.nx * (size_t)p.ny;
  // per-cell-shift storage keeps a tenth plane (the reference density)
  const size_t planes = p.storage == LBM_F16_CELL ? 10 : 9;
  return planes * (size_t)p.nx * (size_t)p.ny * (p.storage == LBM_F32 ? 4 : 2);
}

WorkLayout work_layout(int nx, int ny) {
  WorkLayout w{};
  w.max_items = ((nx + kMinStripWidth - 1) / kMinStripWidth) * ((ny + kMinRows - 1) / kMinRows);
  size_t o = 0;
  w.desc = o;
  o += 256;
  w.nitems = o;
  o += 256;
  w.items = o;
  o = align_up(o + (size_t)w.max_items * sizeof(TileItem), 256);
  w.partials = o;
  o += (size_t)kMaxPartials * kPartialStride * sizeof(double);
  w.result = o;
  o += 256;
  // the series tile: kSeriesThreads-wide strips, row index 0 (8-row bands)
  w.series_items = ((nx + kSeriesThreads - 1) / kSeriesThreads) *
                   ((ny + kRowChoices[0] - 1) / kRowChoices[0]);
  // and the two-step recording tile: strips of series2_width columns (the
  // narrowest, FP32's, sizes the table), kSeries2Rows-row bands
  const int w2 = kSeries2WidthF32;
  w.series2_items = ((nx + w2 - 1) / w2) * ((ny + kSeries2Rows - 1) / kSeries2Rows);
  w.s_nitems = o;
  o += 256;
  w.s_items = o;
  o = align_up(o + (size_t)w.series_items * sizeof(TileItem), 256);
  w.s2_nitems = o;
  o += 256;
  w.s2_items = o;
  o = align_up(o + (size_t)w.series2_items * sizeof(TileItem), 256);
  w.s_partials = o;
  o = align_up(o + (size_t)std::max(w.series_items, w.series2_items) * kPartialStride *
                       sizeof(double), 256);
  w.s_records = o;
  o += (size_t)kSeriesChunk * 16 * sizeof(double);
  w.total = o;
  return w;
}

// Bands alternate their march direction, so the two bands on either side of
// a band boundary reach the rows they share at the same time (both at the
// start or both at the end of their march) and read them once from L2.
void make_items(int nx, int ny, int storage, int tile, int inst, std::vector<TileItem>& out) {
  const int sw = strip_width(tile, nx), rows = band_rows(tile, nx, ny, storage);
  int band = 0;
  for (int y0 = 0; y0 < ny; y0 += rows, ++band)
    for (int x0 = 0; x0 < nx; x0 += sw)
      out.push_back({inst, x0, y0, (int16_t)std::min(rows, ny - y0), (int16_t)(band & 1)});
}

std::vector<TileItem> xcd_order(const std::vector<TileItem>& items) {
  const size_t n = items.size();
  const size_t nx = 8;
  if (n < 2 * nx) return items;
  const size_t chunk = (n + nx - 1) / nx;
  std::vector<TileItem> out;
  out.reserve(n);
  for (size_t local = 0; local < chunk; ++local)
    for (size_t k = 0; k < nx; ++k) {
      const size_t src = k * chunk + local;
      if (local < chunk && src < std::min(n, (k + 1) * chunk)) out.push_back(items[src]);
    }
  return out;
}

// Workgroups of a step variant resident on the whole device at once (looked
// up once per storage type and variant; 4 per CU if the query fails).
static int resident_blocks(int storage, int variant) {
  static std::mutex mu;
  static int known[kNumStorages][kNumVariants] = {};
  std::lock_guard<std::mutex> lk(mu);
  int& r = known[storage][variant];
  if (r == 0) {
    int per_cu = 0;
    if (step_occupancy(storage, variant, &per_cu) != hipSuccess || per_cu < 1) per_cu = 4;
    r = per_cu * device_cu_count();
  }
  return r;
}

int band_rows(int k, int nx, int ny, int storage) {
  const int r = tile_rows(k);
  if (r > 0) return r;
  const int sw = strip_width(k, nx);
  const int strips = (nx + sw - 1) / sw;
  const int bands = std::max(1, kBalancedRounds * resident_blocks(storage, tile_variant(k)) / strips);
  return std::min(std::max((ny + bands - 1) / bands, kMinRows), kMaxBalancedRows);
}

int row_choice(int rows) {
  for (int r = 0; r < kNumRows; ++r)
    if (kRowChoices[r] == rows) return r;
  return 0;
}

// Default shapes from measurements on MI355X: long bands once the grid alone
// fills the GPU (4096^2: 64 rows), short ones when it does not (1024^2: 4
// rows, 512^2 and below: 2 rows); the widest strip the grid can use.
int default_strip_tile(const lbm_params& p) {
  const size_t cells = (size_t)p.nx * (size_t)p.ny;
  const int rows = cells >= (4u << 20) ? 64 : (cells >= (1u << 20) ? 4 : 2);
  int v;
  if (p.storage != LBM_F32 && p.nx > 128)
    v = find_variant(256, 2, 1, 0);  // 512 columns, two cells per thread
  else if (p.nx >= 512)
    v = find_variant(512, 1, 2, 0);
  else if (p.nx >= 256)
    v = find_variant(256, 1, 2, 0);
  else if (p.nx >= 128)
    v = find_variant(128, 1, 2, 0);
  else
    v = find_variant(64, 1, 1, 0);
  return v * kNumRows + row_choice(rows);
}

int default_tile(const lbm_params& p) {
  const size_t cells = (size_t)p.nx * (size_t)p.ny;
  // Moment storage: two steps per launch from a million cells (256 threads
  // writing 240 columns, balanced bands) and on grids up to 512 columns wide
  // (one periodic strip, balanced bands); strips of 256 threads x 1 cell, 2
  // rows in flight, with the band heights of the strip defaults otherwise.
  if (p.storage == LBM_F16_MOMENT) {
    if (cells >= (1u << 20)) return find_variant(256, 1, 1, 0, 2, 240) * kNumRows + row_choice(0);
    if (p.nx <= 512) {
      const int nt = p.nx <= 128 ? 128 : (p.nx <= 256 ? 256 : 512);
      return find_variant(nt, 1, 1, 0, 2, nt - 16) * kNumRows + row_choice(0);  // 112, 240, 496 columns
    }
    return find_variant(256, 1, 2, 0) * kNumRows + default_strip_tile(p) % kNumRows;
  }
  // From a million cells up, FP32 takes three steps per launch: 256 threads
  // writing 240 columns (64-byte-aligned strips) in 32-row bands from 16M
  // cells, 128 threads writing 112 columns below that (32-row bands from 4M
  // cells, 8-row below).  The FP16 forms take two steps per launch: shifted
  // from 16M cells with 256 threads, 2 rows in flight and balanced bands,
  // below that with 128 threads (8-row bands below 4M cells, else balanced);
  // FP16 shifted per cell with 256 threads and 2 rows in flight (balanced
  // bands from 16M cells, 16-row from 4M, 8-row below).
  if (cells >= (1u << 20)) {
    if (p.storage == LBM_F32) {
      if (cells >= (16u << 20)) return find_variant(256, 1, 1, 0, 3, 240) * kNumRows + row_choice(32);
      return find_variant(128, 1, 1, 0, 3, 112) * kNumRows +
             row_choice(cells >= (4u << 20) ? 32 : 8);
    }
    if (p.storage == LBM_F16_SHIFTED && cells >= (16u << 20))
      return find_variant(256, 1, 2, 0, 2) * kNumRows + row_choice(0);
    if (p.storage == LBM_F16_SHIFTED)
      return find_variant(128, 1, 1, 0, 2) * kNumRows + row_choice(cells >= (4u << 20) ? 0 : 8);
    return find_variant(256, 1, 2, 0, 2) * kNumRows +
           row_choice(cells >= (16u << 20) ? 0 : (cells >= (4u << 20) ? 16 : 8));
  }
  // Below a million cells, a grid no wider than a two-step workgroup runs as
  // one periodic strip, two steps per launch, balanced bands: 128 threads up
  // to 128 columns, 256 up to 256, else 512; FP16 per cell with 2 rows in
  // flight and at least 256 threads.
  if (p.nx <= 512) {
    const bool percell = p.storage == LBM_F16_CELL;
    const int nt = p.nx <= 128 && !percell ? 128 : (p.nx <= 256 ? 256 : 512);
    return find_variant(nt, 1, percell ? 2 : 1, 0, 2) * kNumRows + row_choice(0);
  }
  // Below a million cells on grids wider than 512 columns: FP32 three steps
  // per launch (128 threads writing 112 columns, 8-row bands); FP16 storage
  // paired columns, 4 wavefronts, 2 rows in flight, 2-row bands, where the
  // grid allows it.
  if (p.storage == LBM_F32) return find_variant(128, 1, 1, 0, 3, 112) * kNumRows + row_choice(8);
  {
    const int k = find_variant(256, 2, 2, 1) * kNumRows + row_choice(2);
    if (tile_valid(k, p.nx, p.storage)) return k;
  }
  return default_strip_tile(p);
}

// Architecture name of the current device, looked up once per device
// (hipGetDeviceProperties is slow enough to matter per created run).
std::string device_arch() {
  static std::mutex mu;
  static std::map<int, std::string> known;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  std::lock_guard<std::mutex> lk(mu);
  auto it = known.find(dev);
  if (it != known.end()) return it->second;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  a = c == std::string::npos ? a : a.substr(0, c);
  known[dev] = a;
  return a;
}

int device_cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256;
  return cus > 0 ? cus : 256;
}

// ------------------------------------------------------------------ tuning cache
// JSON Lines, one object per (arch, storage, log2-size bucket of nx and ny).

static std::mutex g_tune_mu;

static int size_bucket(int n) {
  int b = 0;
  while ((1 << b) < n) ++b;
  return b;
}

// Each entry also records the size of the tile table it indexes, so entries
// written by a build with other tile shapes are ignored.
struct TuneEntry {
  std::string arch;
  int tiles, storage, bx, by, tile;
  double ms;
};

static std::vector<TuneEntry> read_tune_cache(const char* path) {
  std::vector<TuneEntry> v;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    char arch[64] = {0};
    TuneEntry e{};
    if (sscanf(line.c_str(),
               "{\"arch\": \"%63[^\"]\", \"tiles\": %d, \"storage\": %d, \"bx\": %d, \"by\": %d, "
               "\"tile\": %d, \"ms\": %lf}",
               arch, &e.tiles, &e.storage, &e.bx, &e.by, &e.tile, &e.ms) == 7 &&
        e.tiles == kNumTiles && e.tile >= 0 && e.tile < kNumTiles) {
      e.arch = arch;
      v.push_back(e);
    }
  }
  return v;
}

int tuned_tile(const lbm_params& p, const std::string& arch) {
  const char* path = getenv("SCLBM_TUNE_CACHE");
  if (!path || !*path) return -1;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const int bx = size_bucket(p.nx), by = size_bucket(p.ny);
  for (const TuneEntry& e : read_tune_cache(path))
    if (e.arch == arch && e.storage == p.storage && e.bx == bx && e.by == by) return e.tile;
  return -1;
}

void record_tuned_tile(const lbm_params& p, const std::string& arch, int tile, double ms) {
  const char* path = getenv("SCLBM_TUNE_CACHE");
  if (!path || !*path) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::vector<TuneEntry> v = read_tune_cache(path);
  const int bx = size_bucket(p.nx), by = size_bucket(p.ny);
  v.erase(std::remove_if(v.begin(), v.end(),
                         [&](const TuneEntry& e) {
                           return e.arch == arch && e.storage == p.storage && e.bx == bx &&
                                  e.by == by;
                         }),
          v.end());
  v.push_back({arch, kNumTiles, p.storage, bx, by, tile, ms});
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    for (const TuneEntry& e : v) {
      char buf[256];
      snprintf(buf, sizeof buf,
               "{\"arch\": \"%s\", \"tiles\": %d, \"storage\": %d, \"bx\": %d, \"by\": %d, "
               "\"tile\": %d, \"ms\": %.6f}\n",
               e.arch.c_str(), e.tiles, e.storage, e.bx, e.by, e.tile, e.ms);
      out << buf;
    }
  }
  std::rename(tmp.c_str(), path);
}

}  // namespace sclbm

using namespace sclbm;

// ------------------------------------------------------------------ lbm_ctx

InstDesc lbm_ctx::host_desc() const {
  InstDesc d{};
  d.pop[0] = reinterpret_cast<uint64_t>(pop[0]);
  d.pop[1] = reinterpret_cast<uint64_t>(pop[1]);
  d.nx = p.nx;
  d.ny = p.ny;
  d.G = (float)p.G;
  d.tau = (float)p.tau;
  d.omega = (float)(1.0 / p.tau);
  d.rho0 = p.storage == LBM_F16_SHIFTED ? (float)p.rho0 : 0.0f;
  d.parity = 0;
  d.nsub = INT32_MAX;
  d.storage = p.storage;
  d.flag = reinterpret_cast<uint64_t>(flag);
  return d;
}

lbm_status lbm_ctx::upload_tile(int k) {
  std::vector<TileItem> items;
  make_items(p.nx, p.ny, p.storage, k, 0, items);
  items = xcd_order(items);
  if ((int)items.size() > lay.max_items) return fail(LBM_EINVAL, "tile table overflow");
  const int n = (int)items.size();
  SCLBM_HIP(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(TileItem),
                           hipMemcpyHostToDevice, stream));
  SCLBM_HIP(hipMemcpyAsync(d_nitems, &n, sizeof(int), hipMemcpyHostToDevice, stream));
  SCLBM_HIP(hipStreamSynchronize(stream));
  tile = k;
  nitems = n;
  return LBM_OK;
}

lbm_status lbm_ctx::diagnostics(lbm_metrics* out) {
  if (!h_result)
    SCLBM_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_result), 16 * sizeof(double),
                            hipHostMallocDefault));
  void* idle = pop[parity ^ 1];
  SCLBM_HIP(launch_diagnostics(p.storage, pop[parity], p.nx, p.ny, host_desc().rho0,
                               reinterpret_cast<double*>(idle), d_partials, d_result, stream));
  SCLBM_HIP(hipMemcpyAsync(h_result, d_result, 10 * sizeof(double), hipMemcpyDeviceToHost, stream));
  SCLBM_HIP(hipStreamSynchronize(stream));
  *out = metrics_from_raw(h_result, steps);
  return LBM_OK;
}

// Metrics from the ten raw values {mass, mom_x, mom_y, bad cells, cells above
// the threshold, G_max, sum |grad rho|, sum |grad rho|^2, rho_max, rho_min}:
// Eqs. (9)-(13) with V_total = nx * ny cells.
lbm_metrics lbm_ctx::metrics_from_raw(const double* r, int64_t step) const {
  const double ncell = (double)p.nx * (double)p.ny;
  lbm_metrics m{};
  m.mass = r[0];
  m.mom_x = r[1];
  m.mom_y = r[2];
  m.finite = r[3] == 0.0 ? 1 : 0;
  m.n_above = (int64_t)r[4];
  m.Gmax = r[5];
  m.sum_grad = r[6];
  m.E_int = r[7];
  m.rho_max = r[8];
  m.rho_min = r[9];
  m.W = r[4] / ncell;
  m.drho = r[8] - r[9];
  m.W_eff = r[5] > 0.0 ? r[6] / (r[5] * ncell) : 0.0;
  m.step = step;
  return m;
}

// The series tile tables (built on first use).  Single-step: strips of
// kSeriesThreads x 1 cell, 2 rows in flight, 8-row bands (also the
// single-step tile of runs whose own tile takes two steps per launch).
// Two-step: kSeriesThreads threads, 1 row in flight, kSeries2Rows-row bands.
lbm_status lbm_ctx::series_tiles() {
  if (series_nitems > 0) return LBM_OK;
  auto build = [&](int k, int cap, TileItem* d_it, int* d_n, int* count) -> lbm_status {
    std::vector<TileItem> items;
    make_items(p.nx, p.ny, p.storage, k, 0, items);
    items = xcd_order(items);
    if ((int)items.size() > cap) return fail(LBM_EINVAL, "series tile table overflow");
    *count = (int)items.size();
    SCLBM_HIP(hipMemcpyAsync(d_it, items.data(), items.size() * sizeof(TileItem),
                             hipMemcpyHostToDevice, stream));
    SCLBM_HIP(hipMemcpyAsync(d_n, count, sizeof(int), hipMemcpyHostToDevice, stream));
    return LBM_OK;
  };
  int n1 = 0, n2 = 0;
  lbm_status r = build(find_variant(kSeriesThreads, 1, 2, 0) * kNumRows + row_choice(8),
                       lay.series_items, d_sitems, d_snitems, &n1);
  if (r == LBM_OK)
    r = build(find_variant(kSeriesThreads, 1, 1, 0, 2, series2_width(p.storage)) * kNumRows +
                  row_choice(kSeries2Rows),
              lay.series2_items, d_s2items, d_s2nitems, &n2);
  if (r != LBM_OK) return r;
  SCLBM_HIP(hipStreamSynchronize(stream));
  series_nitems = n1;
  series2_nitems = n2;
  return LBM_OK;
}

// Two-step variant of the same strips as three-step variant v (-1 for others).
static int pair_variant_for(int v) {
  const StepVariant& sv = step_variant(v);
  return sv.steps == 3 ? find_variant(sv.threads, 1, sv.prefetch, 0, 2, sv.width) : -1;
}

lbm_status lbm_ctx::advance(int64_t n) {
  const int v = tile_variant(tile);
  const int per = tile_steps(tile);
  for (; n >= per; n -= per) {
    SCLBM_HIP(launch_step(p.storage, v, d_desc, d_items, d_nitems, nitems, parity, stream));
    parity ^= 1;
    steps += per;
  }
  if (n >= 2) {
    // two steps left after three-step launches: the two-step variant of the
    // same strips, over the same work items
    const int v2 = pair_variant_for(v);
    if (v2 < 0) return fail(LBM_EDEVICE, "no two-step variant for a three-step tile");
    SCLBM_HIP(launch_step(p.storage, v2, d_desc, d_items, d_nitems, nitems, parity, stream));
    parity ^= 1;
    steps += 2;
    n -= 2;
  }
  if (n > 0) {
    const lbm_status s = series_tiles();
    if (s != LBM_OK) return s;
    const int sv = find_variant(kSeriesThreads, 1, 2, 0);
    for (; n > 0; --n) {
      SCLBM_HIP(launch_step(p.storage, sv, d_desc, d_sitems, d_snitems, series_nitems, parity,
                            stream));
      parity ^= 1;
      steps += 1;
    }
  }
  return LBM_OK;
}

lbm_status lbm_ctx::step_series(int64_t n, int32_t every, lbm_metrics* out, int32_t* count) {
  {
    const lbm_status s = series_tiles();
    if (s != LBM_OK) return s;
  }
  if (!h_series)
    SCLBM_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_series),
                            (size_t)kSeriesChunk * 16 * sizeof(double), hipHostMallocDefault));
  int32_t done = 0, pending = 0;
  int64_t first_step = steps;
  auto flush = [&]() -> lbm_status {
    if (pending == 0) return LBM_OK;
    SCLBM_HIP(hipMemcpyAsync(h_series, d_srecords, (size_t)pending * 16 * sizeof(double),
                             hipMemcpyDeviceToHost, stream));
    SCLBM_HIP(hipStreamSynchronize(stream));
    for (int32_t q = 0; q < pending; ++q)
      out[done + q] = metrics_from_raw(h_series + (size_t)q * 16, first_step + (int64_t)q * every);
    done += pending;
    first_step += (int64_t)pending * every;
    pending = 0;
    return LBM_OK;
  };
  for (int64_t j = 0; j < n;) {
    // The step that records the metrics, then the plain steps up to the next
    // record.  With at least one plain step to follow, the recording launch
    // takes two steps (moment storage: always one).
    const int64_t plain = std::min<int64_t>(every - 1, n - j - 1);
    double* rec = d_srecords + (size_t)pending * 16;
    const bool two = plain >= 1 && p.storage != LBM_F16_MOMENT;
    if (two) {
      SCLBM_HIP(launch_step2_diag(p.storage, d_desc, d_s2items, d_s2nitems, series2_nitems,
                                  parity, d_spartials, rec, stream));
      steps += 2;
    } else {
      SCLBM_HIP(launch_step_diag(p.storage, d_desc, d_sitems, d_snitems, series_nitems, parity,
                                 d_spartials, rec, stream));
      steps += 1;
    }
    parity ^= 1;
    if (++pending == kSeriesChunk) {
      const lbm_status s = flush();
      if (s != LBM_OK) return s;
    }
    const lbm_status s = advance(two ? plain - 1 : plain);
    if (s != LBM_OK) return s;
    j += 1 + plain;
  }
  const lbm_status s = flush();
  if (s != LBM_OK) return s;
  *count = done;
  return LBM_OK;
}

// ------------------------------------------------------------------ batch engine

namespace sclbm {
hipError_t graph_add_step(hipGraph_t g, hipGraphNode_t* node, const hipGraphNode_t* deps, size_t nd,
                          int storage, int variant, const InstDesc* descs, const TileItem* items,
                          const int* nitems, int grid, int sub);
hipError_t graph_add_tick(hipGraph_t g, hipGraphNode_t* node, const hipGraphNode_t* deps,
                          size_t nd, bool begin, InstDesc* descs, int n, int K);
hipError_t launch_batch_arm(InstDesc* descs, int n, int64_t steps, hipStream_t st);

size_t BatchEngine::work_bytes(int cap_inst, const int cap_items[kNumStorages],
                               const int cap_titems[kNumStorages], int K) {
  (void)K;
  size_t o = align_up((size_t)cap_inst * sizeof(InstDesc), 256);
  for (int s = 0; s < kNumStorages; ++s) {
    o += 256 + align_up((size_t)cap_items[s] * sizeof(TileItem), 256);
    if (cap_titems[s] > 0) o += 256 + align_up((size_t)cap_titems[s] * sizeof(TileItem), 256);
  }
  return o;
}

int tail_variant_for(int variant) {
  return step_variant(variant).steps >= 2 ? find_variant(kSeriesThreads, 1, 2, 0) : -1;
}


lbm_status BatchEngine::init(hipStream_t st, int steps_per_tick, int cap_inst_,
                             const int cap_items_[kNumStorages],
                             const int cap_titems_[kNumStorages],
                             const int variants[kNumStorages], void* work, size_t wbytes) {
  stream = st;
  K = steps_per_tick;
  cap_inst = cap_inst_;
  if (wbytes < work_bytes(cap_inst, cap_items_, cap_titems_, K))
    return fail(LBM_ENOMEM, "batch workspace too small");
  char* w = reinterpret_cast<char*>(work);
  size_t o = 0;
  d_desc = reinterpret_cast<InstDesc*>(w);
  o = align_up((size_t)cap_inst * sizeof(InstDesc), 256);
  const int cus = device_cu_count();
  // Persistent engines (item counts change between replays) run a grid sized
  // to the resident capacity; fixed ones launch one workgroup per item, so
  // the hardware overlaps one item's tail with the next item's loads.
  auto grid_for = [&](int s, int v, int cap, int* g) -> lbm_status {
    int occ = 0;
    SCLBM_HIP(step_occupancy(s, v, &occ));
    const int res = std::max(8, std::max(occ, 1) * cus / 8 * 8);
    *g = persistent ? std::min(cap, res) : cap;
    return LBM_OK;
  };
  for (int s = 0; s < kNumStorages; ++s) {
    cap_items[s] = cap_items_[s];
    variant[s] = variants[s];
    d_nitems[s] = reinterpret_cast<int*>(w + o);
    o += 256;
    d_items[s] = reinterpret_cast<TileItem*>(w + o);
    o += align_up((size_t)cap_items[s] * sizeof(TileItem), 256);
    grid[s] = tgrid[s] = 0;
    cap_titems[s] = cap_titems_[s];
    tail_variant[s] = pair_variant[s] = -1;
    if (cap_titems[s] > 0) {
      d_tnitems[s] = reinterpret_cast<int*>(w + o);
      o += 256;
      d_titems[s] = reinterpret_cast<TileItem*>(w + o);
      o += align_up((size_t)cap_titems[s] * sizeof(TileItem), 256);
    }
    if (variant[s] < 0 || cap_items[s] == 0) continue;
    lbm_status r = grid_for(s, variant[s], cap_items[s], &grid[s]);
    if (r != LBM_OK) return r;
    if (per_launch(s) >= 2) {
      if (cap_titems[s] == 0) return fail(LBM_EINVAL, "multi-step batch without a tail table");
      tail_variant[s] = tail_variant_for(variant[s]);
      r = grid_for(s, tail_variant[s], cap_titems[s], &tgrid[s]);
      if (r != LBM_OK) return r;
    }
    if (per_launch(s) == 3) {
      pair_variant[s] = pair_variant_for(variant[s]);
      if (pair_variant[s] < 0) return fail(LBM_EINVAL, "no two-step variant for a three-step batch");
      r = grid_for(s, pair_variant[s], cap_items[s], &p2grid[s]);
      if (r != LBM_OK) return r;
    }
  }
  for (int b = 0; b < 2; ++b)
    SCLBM_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_desc[b]),
                            (size_t)cap_inst * sizeof(InstDesc), hipHostMallocDefault));
  for (int s = 0; s < kNumStorages; ++s)
    for (int b = 0; b < 2; ++b) {
      if (cap_items[s] > 0)
        SCLBM_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_items[s][b]),
                                (size_t)cap_items[s] * sizeof(TileItem) + 64,
                                hipHostMallocDefault));
      if (cap_titems[s] > 0)
        SCLBM_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_titems[s][b]),
                                (size_t)cap_titems[s] * sizeof(TileItem) + 64,
                                hipHostMallocDefault));
    }
  for (int b = 0; b < 2; ++b)
    SCLBM_HIP(hipEventCreateWithFlags(&staged[b], hipEventDisableTiming));
  // Graph: tick_begin -> the step launches of every storage type (K single
  // steps; ceil(K / 2) two-step launches and a tail; or floor(K / 3)
  // three-step launches and two tails) -> tick_end.
  SCLBM_HIP(hipGraphCreate(&graph, 0));
  hipGraphNode_t prev;
  SCLBM_HIP(graph_add_tick(graph, &prev, nullptr, 0, true, d_desc, cap_inst, K));
  int launches[kNumStorages], most = 0;
  for (int s = 0; s < kNumStorages; ++s) {
    const int per = per_launch(s);
    launches[s] = grid[s] == 0 ? 0 : (per == 3 ? K / 3 : (per == 2 ? (K + 1) / 2 : K));
    most = std::max(most, launches[s]);
  }
  for (int j = 0; j < most; ++j)
    for (int s = 0; s < kNumStorages; ++s) {
      if (j >= launches[s]) continue;
      hipGraphNode_t node;
      SCLBM_HIP(graph_add_step(graph, &node, &prev, 1, s, variant[s], d_desc, d_items[s],
                               d_nitems[s], grid[s], j));
      step_nodes[s].push_back(node);
      prev = node;
    }
  for (int s = 0; s < kNumStorages; ++s) {
    if (grid[s] == 0 || per_launch(s) != 3) continue;
    hipGraphNode_t node;
    SCLBM_HIP(graph_add_step(graph, &node, &prev, 1, s, pair_variant[s], d_desc, d_items[s],
                             d_nitems[s], p2grid[s], kTail2Sub));
    step_nodes[s].push_back(node);
    prev = node;
  }
  for (int s = 0; s < kNumStorages; ++s) {
    if (grid[s] == 0 || per_launch(s) < 2) continue;
    hipGraphNode_t node;
    SCLBM_HIP(graph_add_step(graph, &node, &prev, 1, s, tail_variant[s], d_desc, d_titems[s],
                             d_tnitems[s], tgrid[s], kTailSub));
    step_nodes[s].push_back(node);
    prev = node;
  }
  hipGraphNode_t last;
  SCLBM_HIP(graph_add_tick(graph, &last, &prev, 1, false, d_desc, cap_inst, K));
  SCLBM_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  for (int s = 0; s < kNumStorages; ++s) {
    enabled[s] = !lazy_storages;
    if (lazy_storages)
      for (hipGraphNode_t n : step_nodes[s]) SCLBM_HIP(hipGraphNodeSetEnabled(exec, n, 0));
  }
  return LBM_OK;
}

lbm_status BatchEngine::load(const std::vector<lbm_ctx*>& m, const std::vector<int64_t>& remaining,
                             int nsub_init) {
  if ((int)m.size() > cap_inst) return fail(LBM_EINVAL, "too many batch members");
  // Two sets of staging buffers alternate: this load may reuse a set only
  // once the upload that last read it has run.
  const int sb = stage;
  stage ^= 1;
  if (staged_pending[sb]) SCLBM_HIP(hipEventSynchronize(staged[sb]));
  InstDesc* hd = h_desc[sb];
  int count[kNumStorages] = {}, tcount[kNumStorages] = {};
  for (int i = 0; i < cap_inst; ++i) {
    InstDesc d{};
    d.nsub = 0;
    if (i < (int)m.size()) {
      lbm_ctx* c = m[i];
      d = c->host_desc();
      d.parity = c->parity;
      d.nsub = nsub_init;
      d.remaining = remaining[i];
      d.steps = c->steps;
      const int s = c->p.storage;
      if (grid[s] == 0) return fail(LBM_EINVAL, "batch has no kernel for this storage type");
      d.per_launch = per_launch(s);
      const int k = member_tile(c, variant[s], tile_override, row_override);
      std::vector<TileItem> items;
      make_items(c->p.nx, c->p.ny, s, k, i, items);
      if (count[s] + (int)items.size() > cap_items[s])
        return fail(LBM_ENOMEM, "batch tile table full");
      std::copy(items.begin(), items.end(), h_items[s][sb] + count[s]);
      count[s] += (int)items.size();
      if (d.per_launch >= 2) {  // the tail launch's items: same band height
        items.clear();
        make_items(c->p.nx, c->p.ny, s, tail_variant[s] * kNumRows + k % kNumRows, i, items);
        if (tcount[s] + (int)items.size() > cap_titems[s])
          return fail(LBM_ENOMEM, "batch tile table full");
        std::copy(items.begin(), items.end(), h_titems[s][sb] + tcount[s]);
        tcount[s] += (int)items.size();
      }
    }
    hd[i] = d;
  }
  // A storage type's launches are enabled with its first members, with no
  // replay in flight (so none already queued sees the change).
  for (int s = 0; s < kNumStorages; ++s) {
    if (enabled[s] || count[s] == 0) continue;
    SCLBM_HIP(hipStreamSynchronize(stream));
    for (hipGraphNode_t n : step_nodes[s]) SCLBM_HIP(hipGraphNodeSetEnabled(exec, n, 1));
    enabled[s] = true;
  }
  SCLBM_HIP(hipMemcpyAsync(d_desc, hd, (size_t)cap_inst * sizeof(InstDesc),
                           hipMemcpyHostToDevice, stream));
  auto upload = [&](TileItem* hi, int cap, int n, TileItem* d_it, int* d_n) -> lbm_status {
    std::vector<TileItem> v(hi, hi + n);
    v = xcd_order(v);
    std::copy(v.begin(), v.end(), hi);
    int* hn = reinterpret_cast<int*>(hi + cap);
    *hn = n;
    if (n > 0)
      SCLBM_HIP(hipMemcpyAsync(d_it, hi, (size_t)n * sizeof(TileItem), hipMemcpyHostToDevice,
                               stream));
    SCLBM_HIP(hipMemcpyAsync(d_n, hn, sizeof(int), hipMemcpyHostToDevice, stream));
    return LBM_OK;
  };
  for (int s = 0; s < kNumStorages; ++s) {
    if (cap_items[s] == 0) continue;
    nitems[s] = count[s];
    lbm_status r = upload(h_items[s][sb], cap_items[s], count[s], d_items[s], d_nitems[s]);
    if (r == LBM_OK && cap_titems[s] > 0)
      r = upload(h_titems[s][sb], cap_titems[s], tcount[s], d_titems[s], d_tnitems[s]);
    if (r != LBM_OK) return r;
  }
  SCLBM_HIP(hipEventRecord(staged[sb], stream));
  staged_pending[sb] = true;
  members = m;
  return LBM_OK;
}

lbm_status BatchEngine::arm(int64_t steps) {
  SCLBM_HIP(launch_batch_arm(d_desc, (int)members.size(), steps, stream));
  return LBM_OK;
}

lbm_status BatchEngine::replay() {
  SCLBM_HIP(hipGraphLaunch(exec, stream));
  return LBM_OK;
}

void BatchEngine::destroy() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  for (int b = 0; b < 2; ++b) {
    if (staged[b]) (void)hipEventDestroy(staged[b]);
    if (h_desc[b]) (void)hipHostFree(h_desc[b]);
    staged[b] = nullptr;
    h_desc[b] = nullptr;
    staged_pending[b] = false;
  }
  for (int s = 0; s < kNumStorages; ++s)
    for (int b = 0; b < 2; ++b) {
      if (h_items[s][b]) (void)hipHostFree(h_items[s][b]);
      if (h_titems[s][b]) (void)hipHostFree(h_titems[s][b]);
      h_items[s][b] = h_titems[s][b] = nullptr;
    }
  exec = nullptr;
  graph = nullptr;
  for (int s = 0; s < kNumStorages; ++s) {
    step_nodes[s].clear();
    enabled[s] = false;
  }
}

// Tile a member uses inside a batch: the batch's override if set, else the
// batch's strip variant with the batch's band height if set, else the
// member's own.
int member_tile(const lbm_ctx* c, int variant, int tile_override, int row_override) {
  if (tile_override >= 0) return tile_override;
  return variant * kNumRows + (row_override >= 0 ? row_override : c->tile % kNumRows);
}

// Step variant used for one storage type: that of the widest member's tile.
// A paired-column variant is kept only if every member of that storage type
// can run it; otherwise the widest member's default strip variant is used.
int pick_variant(const std::vector<lbm_ctx*>& m, int storage) {
  int best = -1, bestn = -1;
  const lbm_ctx* widest = nullptr;
  for (lbm_ctx* c : m)
    if (c->p.storage == storage && c->p.nx > bestn) {
      bestn = c->p.nx;
      best = tile_variant(c->tile);
      widest = c;
    }
  if (best < 0) return best;
  for (lbm_ctx* c : m)
    if (c->p.storage == storage && !tile_batchable(best * kNumRows, c->p.nx, storage))
      return tile_variant(default_strip_tile(widest->p));
  return best;
}

int count_items(const std::vector<lbm_ctx*>& m, int storage, int variant, int tile_override,
                bool tail) {
  int n = 0;
  for (lbm_ctx* c : m) {
    if (c->p.storage != storage) continue;
    int k = member_tile(c, variant, tile_override);  // as make_items tiles it
    if (tail) k = tail_variant_for(variant) * kNumRows + k % kNumRows;
    const int sw = strip_width(k, c->p.nx);
    const int rows = band_rows(k, c->p.nx, c->p.ny, storage);
    n += ((c->p.nx + sw - 1) / sw) * ((c->p.ny + rows - 1) / rows);
  }
  return n;
}

}  // namespace sclbm

struct lbm_batch {
  std::vector<lbm_ctx*> members;
  BatchEngine eng;
  void* work = nullptr;
  size_t work_bytes = 0;
  int K = 1;
};

namespace {

struct BatchShape {
  int variants[kNumStorages];
  int items[kNumStorages];
  int titems[kNumStorages];  // tail items of two-step variants
};

BatchShape batch_shape(const std::vector<lbm_ctx*>& m, int tile_override = -1) {
  BatchShape b{};
  for (int s = 0; s < kNumStorages; ++s) {
    b.variants[s] = pick_variant(m, s);
    if (b.variants[s] >= 0 && tile_override >= 0) b.variants[s] = tile_variant(tile_override);
    const bool used = b.variants[s] >= 0;
    b.items[s] = used ? count_items(m, s, b.variants[s], tile_override) : 0;
    b.titems[s] = used && step_variant(b.variants[s]).steps >= 2
                      ? count_items(m, s, b.variants[s], tile_override, true)
                      : 0;
  }
  return b;
}

// Rebuilds a batch's engine for a tile override (-1: members' own tiles).
lbm_status batch_rebuild(lbm_batch* b, int tile_override, int nsub_init) {
  SCLBM_HIP(hipStreamSynchronize(b->eng.stream));
  hipStream_t st = b->eng.stream;
  b->eng.destroy();
  b->eng = BatchEngine();
  b->eng.tile_override = tile_override;
  const BatchShape shape = batch_shape(b->members, tile_override);
  lbm_status r = b->eng.init(st, b->K, (int)b->members.size(), shape.items, shape.titems,
                             shape.variants, b->work, b->work_bytes);
  if (r == LBM_OK) r = b->eng.load(b->members, std::vector<int64_t>(b->members.size(), 0), nsub_init);
  return r;
}

// Largest item counts over every tile shape the members can run.
BatchShape batch_shape_max(const std::vector<lbm_ctx*>& m) {
  BatchShape b = batch_shape(m);
  for (int k = 0; k < kNumTiles; ++k) {
    bool valid = true;
    for (lbm_ctx* c : m) valid = valid && tile_batchable(k, c->p.nx, c->p.storage);
    if (!valid) continue;
    const BatchShape t = batch_shape(m, k);
    for (int s = 0; s < kNumStorages; ++s) {
      b.items[s] = std::max(b.items[s], t.items[s]);
      b.titems[s] = std::max(b.titems[s], t.titems[s]);
    }
  }
  return b;
}

}  // namespace

// ------------------------------------------------------------------ C-ABI

// standalone = false: a run driven only by a batch engine (the server's
// continuous policy), which keeps its own descriptor and tile tables; the
// run's own are not uploaded, so creating it does not wait for the stream.
lbm_status sclbm::create_ctx(const lbm_params* p, void* popA, void* popB, size_t pop_bytes,
                             void* work, size_t work_bytes, void* hip_stream, bool standalone,
                             lbm_ctx** out, int* flag) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status s = validate_params(p);
  if (s != LBM_OK) return s;
  if (!popA || !popB || !work) return fail(LBM_EINVAL, "buffer pointer is NULL");
  if (popA == popB) return fail(LBM_EINVAL, "popA and popB must be distinct buffers");
  if (((uintptr_t)popA | (uintptr_t)popB | (uintptr_t)work) & 255)
    return fail(LBM_EINVAL, "buffers must be 256-byte aligned");
  const WorkLayout lay = work_layout(p->nx, p->ny);
  if (pop_bytes < pop_bytes_for(*p)) return fail(LBM_ENOMEM, "population buffers too small");
  if (work_bytes < lay.total) return fail(LBM_ENOMEM, "workspace too small");
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_ENOMEM, "host allocation failed");
  c->p = *p;
  c->pop[0] = popA;
  c->pop[1] = popB;
  c->pop_bytes = pop_bytes;
  c->work = work;
  c->work_bytes = work_bytes;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->flag = flag;
  c->lay = lay;
  char* w = reinterpret_cast<char*>(work);
  c->d_desc = reinterpret_cast<InstDesc*>(w + lay.desc);
  c->d_nitems = reinterpret_cast<int*>(w + lay.nitems);
  c->d_items = reinterpret_cast<TileItem*>(w + lay.items);
  c->d_partials = reinterpret_cast<double*>(w + lay.partials);
  c->d_result = reinterpret_cast<double*>(w + lay.result);
  c->d_snitems = reinterpret_cast<int*>(w + lay.s_nitems);
  c->d_sitems = reinterpret_cast<TileItem*>(w + lay.s_items);
  c->d_s2nitems = reinterpret_cast<int*>(w + lay.s2_nitems);
  c->d_s2items = reinterpret_cast<TileItem*>(w + lay.s2_items);
  c->d_spartials = reinterpret_cast<double*>(w + lay.s_partials);
  c->d_srecords = reinterpret_cast<double*>(w + lay.s_records);
  c->arch = device_arch();
  if (!standalone) {
    c->tile = default_tile(*p);  // its band height is what a batch may use
    *out = c;
    return LBM_OK;
  }
  const InstDesc d = c->host_desc();
  hipError_t e = hipMemcpyAsync(c->d_desc, &d, sizeof d, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "descriptor upload");
  }
  int k = tuned_tile(*p, c->arch);
  if (k < 0 || !tile_valid(k, p->nx, p->storage)) k = default_tile(*p);
  s = c->upload_tile(k);
  if (s != LBM_OK) {
    delete c;
    return s;
  }
  *out = c;
  return LBM_OK;
}

// sync = false: returns after enqueueing; the caller keeps `drops` alive
// until the stream has passed the initialisation.
lbm_status sclbm::init_droplets(lbm_ctx* c, const double* drops, int32_t n, const lbm_init* ip,
                                bool sync) {
  if (!c || !ip) return fail(LBM_EINVAL, "ctx or init is NULL");
  if (c->batch) return fail(LBM_EBUSY, "context is a member of a live batch");
  if (n < 0 || (n > 0 && !drops)) return fail(LBM_EINVAL, "bad droplet array");
  const double vals[4] = {ip->rho_l, ip->rho_g, ip->width, ip->noise_amp};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(LBM_EINVAL, "init fields must be finite");
  if (!(ip->width > 0.0) || ip->noise_amp < 0.0)
    return fail(LBM_EINVAL, "width must be > 0 and noise_amp >= 0");
  for (int32_t k = 0; k < 3 * n; ++k)
    if (!std::isfinite(drops[k])) return fail(LBM_EINVAL, "droplet values must be finite");
  InitArgs a{};
  a.nx = c->p.nx;
  a.ny = c->p.ny;
  a.rho_l = ip->rho_l;
  a.rho_g = ip->rho_g;
  a.width = ip->width;
  a.noise_amp = ip->noise_amp;
  a.seed = ip->seed;
  a.period_x = ip->period_x > 0 ? ip->period_x : c->p.nx;
  a.period_y = ip->period_y > 0 ? ip->period_y : c->p.ny;
  a.origin_x = ip->origin_x;
  a.origin_y = ip->origin_y;
  if (ip->period_x < 0 || ip->period_y < 0 || ip->origin_x < 0 || ip->origin_y < 0)
    return fail(LBM_EINVAL, "period and origin must be >= 0");
  if ((ip->period_x == 0 && ip->origin_x != 0) || (ip->period_y == 0 && ip->origin_y != 0))
    return fail(LBM_EINVAL, "origin requires an explicit period");
  if (a.origin_x + c->p.nx > a.period_x || a.origin_y + c->p.ny > a.period_y)
    return fail(LBM_EINVAL, "the grid must lie inside the frame: origin + n <= period");
  // Scratch in the second buffer: rho (FP64) then the droplet list.
  const size_t ncell = (size_t)c->p.nx * c->p.ny;
  const size_t drop_off = align_up(ncell * sizeof(double), 256);
  const size_t cap = c->pop_bytes > drop_off ? (c->pop_bytes - drop_off) / (3 * sizeof(double)) : 0;
  if ((size_t)n > cap)
    return fail(LBM_EINVAL, "too many droplets for this grid's scratch space (max " +
                                std::to_string(cap) + ")");
  char* scratch = reinterpret_cast<char*>(c->pop[1]);
  double* rho64 = reinterpret_cast<double*>(scratch);
  double* d_drops = reinterpret_cast<double*>(scratch + drop_off);
  if (n > 0)
    SCLBM_HIP(hipMemcpyAsync(d_drops, drops, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
  SCLBM_HIP(launch_init(c->p.storage, d_drops, n, a, rho64, c->host_desc().rho0, c->pop[0],
                        c->stream));
  if (sync) SCLBM_HIP(hipStreamSynchronize(c->stream));
  c->parity = 0;
  c->steps = 0;
  return LBM_OK;
}

extern "C" {

const char* lbm_last_error(void) { return g_error.c_str(); }

const char* lbm_version(void) { return "sclbm 0.1 (gfx950)"; }

lbm_status lbm_buffer_bytes(const lbm_params* p, size_t* pop_bytes, size_t* work_bytes) {
  return guarded("lbm_buffer_bytes", [&]() -> lbm_status {
    const lbm_status s = validate_params(p);
    if (s != LBM_OK) return s;
    if (pop_bytes) *pop_bytes = pop_bytes_for(*p);
    if (work_bytes) *work_bytes = work_layout(p->nx, p->ny).total;
    return LBM_OK;
  });
}

lbm_status lbm_create(const lbm_params* p, void* popA, void* popB, size_t pop_bytes, void* work,
                      size_t work_bytes, void* hip_stream, lbm_ctx** out) {
  return guarded("lbm_create", [&]() -> lbm_status {
    return sclbm::create_ctx(p, popA, popB, pop_bytes, work, work_bytes, hip_stream, true, out);
  });
}

lbm_status lbm_destroy(lbm_ctx* c) {
  return guarded("lbm_destroy", [&]() -> lbm_status {
    if (!c) return LBM_OK;
    if (c->batch) return fail(LBM_EBUSY, "context is a member of a live batch");
    const hipError_t e = hipStreamSynchronize(c->stream);
    if (c->h_result) (void)hipHostFree(c->h_result);
    if (c->h_series) (void)hipHostFree(c->h_series);
    delete c;
    return e == hipSuccess ? LBM_OK : hip_fail(e, "hipStreamSynchronize");
  });
}

lbm_status lbm_init_droplets(lbm_ctx* c, const double* drops, int32_t n, const lbm_init* ip) {
  return guarded("lbm_init_droplets", [&]() -> lbm_status {
    return sclbm::init_droplets(c, drops, n, ip, true);
  });
}

lbm_status lbm_step_n(lbm_ctx* c, int64_t n) {
  return guarded("lbm_step_n", [&]() -> lbm_status {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (c->batch) return fail(LBM_EBUSY, "context is a member of a live batch");
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    return c->advance(n);
  });
}

lbm_status lbm_step_series(lbm_ctx* c, int64_t n, int32_t every, lbm_metrics* out,
                           int32_t capacity, int32_t* count) {
  return guarded("lbm_step_series", [&]() -> lbm_status {
    if (!c || !count) return fail(LBM_EINVAL, "ctx or count is NULL");
    *count = 0;
    if (c->batch) return fail(LBM_EBUSY, "context is a member of a live batch");
    if (n < 0 || every < 1) return fail(LBM_EINVAL, "need n >= 0 and every >= 1");
    const int64_t need = (n + every - 1) / every;
    if (need > capacity || (need > 0 && !out))
      return fail(LBM_EINVAL, "out holds fewer than ceil(n / every) records");
    return c->step_series(n, every, out, count);
  });
}

lbm_status lbm_moments(lbm_ctx* c, float* rho, float* ux, float* uy) {
  return guarded("lbm_moments", [&]() -> lbm_status {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!rho && !ux && !uy) return LBM_OK;
    float* r = rho ? rho : reinterpret_cast<float*>(c->pop[c->parity ^ 1]);
    SCLBM_HIP(launch_moments(c->p.storage, c->pop[c->parity], c->p.nx, c->p.ny, c->host_desc().rho0,
                             (float)c->p.G, r, ux, uy, c->stream));
    return LBM_OK;
  });
}

lbm_status lbm_interface_metrics(lbm_ctx* c, lbm_metrics* out) {
  return guarded("lbm_interface_metrics", [&]() -> lbm_status {
    if (!c || !out) return fail(LBM_EINVAL, "ctx or out is NULL");
    return c->diagnostics(out);
  });
}

lbm_status lbm_get_state(lbm_ctx* c, float* f) {
  return guarded("lbm_get_state", [&]() -> lbm_status {
    if (!c || !f) return fail(LBM_EINVAL, "ctx or buffer is NULL");
    SCLBM_HIP(launch_get_state(c->p.storage, c->pop[c->parity], c->p.nx, c->p.ny,
                               c->host_desc().rho0, f, c->stream));
    return LBM_OK;
  });
}

lbm_status lbm_set_state(lbm_ctx* c, const float* f) {
  return guarded("lbm_set_state", [&]() -> lbm_status {
    if (!c || !f) return fail(LBM_EINVAL, "ctx or buffer is NULL");
    if (c->batch) return fail(LBM_EBUSY, "context is a member of a live batch");
    SCLBM_HIP(launch_set_state(c->p.storage, f, c->p.nx, c->p.ny, c->host_desc().rho0,
                               c->pop[c->parity], c->stream));
    return LBM_OK;
  });
}

int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->steps : -1; }

int32_t lbm_tile_count(void) { return kNumTiles; }

lbm_status lbm_tile_describe(int32_t k, int32_t* width, int32_t* rows, int32_t* threads,
                             int32_t* prefetch, int32_t* cells, int32_t* paired, int32_t* steps) {
  return guarded("lbm_tile_describe", [&]() -> lbm_status {
    if (k < 0 || k >= kNumTiles) return fail(LBM_EINVAL, "tile index out of range");
    const StepVariant& v = step_variant(tile_variant(k));
    if (width) *width = tile_width(k);
    if (rows) *rows = tile_rows(k);
    if (threads) *threads = v.threads;
    if (prefetch) *prefetch = v.prefetch;
    if (cells) *cells = v.cells;
    if (paired) *paired = v.paired;
    if (steps) *steps = v.steps;
    return LBM_OK;
  });
}

lbm_status lbm_default_tile(const lbm_params* p, int32_t* k) {
  return guarded("lbm_default_tile", [&]() -> lbm_status {
    const lbm_status v = validate_params(p);
    if (v != LBM_OK) return v;
    if (!k) return fail(LBM_EINVAL, "k is NULL");
    *k = default_tile(*p);
    return LBM_OK;
  });
}

lbm_status lbm_tile_layout(const lbm_params* p, int32_t k, int32_t* rows, int32_t* items) {
  return guarded("lbm_tile_layout", [&]() -> lbm_status {
    const lbm_status v = validate_params(p);
    if (v != LBM_OK) return v;
    if (k < 0 || k >= kNumTiles) return fail(LBM_EINVAL, "tile index out of range");
    const int r = band_rows(k, p->nx, p->ny, p->storage);
    const int w = strip_width(k, p->nx);
    if (rows) *rows = r;
    if (items) *items = ((p->nx + w - 1) / w) * ((p->ny + r - 1) / r);
    return LBM_OK;
  });
}

lbm_status lbm_set_tile(lbm_ctx* c, int32_t k) {
  return guarded("lbm_set_tile", [&]() -> lbm_status {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (k < 0 || k >= kNumTiles) return fail(LBM_EINVAL, "tile index out of range");
    if (!tile_valid(k, c->p.nx, c->p.storage))
      return fail(LBM_EINVAL,
                  c->p.storage == LBM_F16_MOMENT
                      ? "moment storage runs strip shapes and two-step shapes of at most threads - 8 columns"
                  : tile_steps(k) >= 3 ? "three-step tile shapes take FP32 storage only"
                                       : "paired-column tile shapes need an even nx >= 128");
    if (c->batch) return fail(LBM_EBUSY, "context is a member of a live batch");
    return c->upload_tile(k);
  });
}

int32_t lbm_get_tile(const lbm_ctx* c) { return c ? c->tile : -1; }

// Times every valid tile shape on c's grid and selects the fastest per time
// step.  Without scratch, `reps` launches per shape read the current buffer
// and write the idle one (the state is untouched).  With scratch (>= the
// state's bytes) the state is copied there first, each shape advances the run
// as stepping does (every launch reads what the previous one wrote), and the
// state, its buffer and the step count are restored afterwards.
static lbm_status autotune_run(lbm_ctx* c, int32_t reps, void* scratch, int32_t* best_out) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (c->batch) return fail(LBM_EBUSY, "context is a member of a live batch");
  if (reps < 1) return fail(LBM_EINVAL, "reps must be >= 1");
  const size_t state_bytes = pop_bytes_for(c->p);
  const int parity0 = c->parity;
  const int64_t steps0 = c->steps;
  if (scratch)
    SCLBM_HIP(hipMemcpyAsync(scratch, c->pop[parity0], state_bytes, hipMemcpyDeviceToDevice,
                             c->stream));
  hipEvent_t e0, e1;
  SCLBM_HIP(hipEventCreate(&e0));
  SCLBM_HIP(hipEventCreate(&e1));
  int best = c->tile;
  double best_ms = 1e300;
  lbm_status st = LBM_OK;
  for (int k = 0; k < kNumTiles && st == LBM_OK; ++k) {
    if (!tile_valid(k, c->p.nx, c->p.storage)) continue;
    st = c->upload_tile(k);
    if (st != LBM_OK) break;
    const int v = tile_variant(k);
    const int per = tile_steps(k);
    hipError_t e = hipSuccess;
    if (scratch) {
      st = c->advance(per);  // the first launch of the shape, untimed
      if (st == LBM_OK) e = hipEventRecord(e0, c->stream);
      if (st == LBM_OK && e == hipSuccess) st = c->advance((int64_t)reps * per);
      if (st != LBM_OK) break;
    } else {
      // Read the current buffer and write the idle one, leaving the state as is.
      e = launch_step(c->p.storage, v, c->d_desc, c->d_items, c->d_nitems, c->nitems, c->parity,
                      c->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r)
        e = launch_step(c->p.storage, v, c->d_desc, c->d_items, c->d_nitems, c->nitems,
                        c->parity, c->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      st = hip_fail(e, "autotune launch");
      break;
    }
    const double per_step = ms / reps / per;
    if (per_step < best_ms) {
      best_ms = per_step;
      best = k;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (scratch) {
    // the state back in the buffer it started in, whatever the loop reached
    c->parity = parity0;
    c->steps = steps0;
    const hipError_t e = hipMemcpyAsync(c->pop[parity0], scratch, state_bytes,
                                        hipMemcpyDeviceToDevice, c->stream);
    if (st == LBM_OK && e != hipSuccess) st = hip_fail(e, "autotune restore");
    const hipError_t e2 = hipStreamSynchronize(c->stream);
    if (st == LBM_OK && e2 != hipSuccess) st = hip_fail(e2, "hipStreamSynchronize");
  }
  if (st != LBM_OK) return st;
  st = c->upload_tile(best);
  if (st != LBM_OK) return st;
  record_tuned_tile(c->p, c->arch, best, best_ms);
  if (best_out) *best_out = best;
  return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx* c, int32_t reps, int32_t* best_out) {
  return guarded("lbm_autotune",
                 [&]() -> lbm_status { return autotune_run(c, reps, nullptr, best_out); });
}

lbm_status lbm_autotune_stepping(lbm_ctx* c, int32_t reps, void* scratch, size_t scratch_bytes,
                                 int32_t* best_out) {
  return guarded("lbm_autotune_stepping", [&]() -> lbm_status {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!scratch) return fail(LBM_EINVAL, "scratch is NULL");
    if ((uintptr_t)scratch & 255) return fail(LBM_EINVAL, "scratch must be 256-byte aligned");
    if (scratch_bytes < pop_bytes_for(c->p)) return fail(LBM_ENOMEM, "scratch smaller than the state");
    return autotune_run(c, reps, scratch, best_out);
  });
}

// ------------------------------------------------------------------ batch C-ABI

lbm_status lbm_batch_work_bytes(lbm_ctx* const* ctxs, int32_t n, size_t* bytes) {
  return guarded("lbm_batch_work_bytes", [&]() -> lbm_status {
    if (!ctxs || n < 1 || !bytes) return fail(LBM_EINVAL, "bad batch arguments");
    std::vector<lbm_ctx*> m(ctxs, ctxs + n);
    for (lbm_ctx* c : m)
      if (!c) return fail(LBM_EINVAL, "NULL context in batch");
    const BatchShape b = batch_shape_max(m);
    *bytes = BatchEngine::work_bytes(n, b.items, b.titems, kMaxGraphSteps);
    return LBM_OK;
  });
}

lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int32_t n, void* work, size_t work_bytes,
                            int32_t steps_per_graph, lbm_batch** out) {
  return guarded("lbm_batch_create", [&]() -> lbm_status {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctxs || n < 1 || !work) return fail(LBM_EINVAL, "bad batch arguments");
    if (steps_per_graph < 1 || steps_per_graph > kMaxGraphSteps)
      return fail(LBM_EINVAL, "steps_per_graph must be in [1, " + std::to_string(kMaxGraphSteps) + "]");
    if ((uintptr_t)work & 255) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    std::vector<lbm_ctx*> m(ctxs, ctxs + n);
    for (size_t i = 0; i < m.size(); ++i) {
      if (!m[i]) return fail(LBM_EINVAL, "NULL context in batch");
      if (m[i]->batch) return fail(LBM_EBUSY, "context already belongs to a batch");
      if (m[i]->stream != m[0]->stream) return fail(LBM_EINVAL, "batch members need one stream");
      for (size_t j = 0; j < i; ++j)
        if (m[j] == m[i]) return fail(LBM_EINVAL, "context listed twice");
    }
    const BatchShape shape = batch_shape(m);
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_ENOMEM, "host allocation failed");
    b->members = m;
    b->work = work;
    b->work_bytes = work_bytes;
    b->K = steps_per_graph;
    lbm_status st = b->eng.init(m[0]->stream, steps_per_graph, n, shape.items, shape.titems,
                                shape.variants, work, work_bytes);
    if (st == LBM_OK) st = b->eng.load(m, std::vector<int64_t>(m.size(), 0));
    if (st != LBM_OK) {
      b->eng.destroy();
      delete b;
      return st;
    }
    for (lbm_ctx* c : m) c->batch = b;
    *out = b;
    return LBM_OK;
  });
}

lbm_status lbm_batch_step_n(lbm_batch* b, int64_t n) {
  return guarded("lbm_batch_step_n", [&]() -> lbm_status {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    if (n == 0) return LBM_OK;
    lbm_status st = b->eng.arm(n);
    const int64_t replays = (n + b->eng.K - 1) / b->eng.K;
    for (int64_t r = 0; r < replays && st == LBM_OK; ++r) st = b->eng.replay();
    if (st != LBM_OK) return st;
    const int64_t K = b->eng.K;
    for (lbm_ctx* c : b->members) {
      const int per = b->eng.per_launch(c->p.storage);
      const int64_t flips = (n / K) * tick_flips(K, per) + tick_flips(n % K, per);
      c->steps += n;
      c->parity = (int)((c->parity + flips) & 1);
    }
    return LBM_OK;
  });
}

lbm_status lbm_batch_autotune(lbm_batch* b, int32_t reps, int32_t* best_out) {
  return guarded("lbm_batch_autotune", [&]() -> lbm_status {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (reps < 1) return fail(LBM_EINVAL, "reps must be >= 1");
    hipEvent_t e0, e1;
    SCLBM_HIP(hipEventCreate(&e0));
    SCLBM_HIP(hipEventCreate(&e1));
    int best = -1;
    double best_ms = 1e300;
    lbm_status st = LBM_OK;
    for (int k = 0; k < kNumTiles && st == LBM_OK; ++k) {
      bool valid = true;
      for (lbm_ctx* c : b->members) valid = valid && tile_batchable(k, c->p.nx, c->p.storage);
      if (!valid) continue;
      // Every member takes one launch (of one, two or three steps) from
      // its current buffer into its idle one, and the descriptors are not
      // advanced: the state is unchanged.  Compared per time step.
      const int per = tile_steps(k);
      st = batch_rebuild(b, k, per);
      if (st == LBM_ENOMEM) {  // this shape's tables do not fit the workspace
        st = LBM_OK;
        continue;
      }
      if (st != LBM_OK) break;
      BatchEngine& g = b->eng;
      auto launch_all = [&]() {
        hipError_t e = hipSuccess;
        for (int s = 0; s < kNumStorages && e == hipSuccess; ++s)
          if (g.grid[s] > 0)
            e = launch_step(s, g.variant[s], g.d_desc, g.d_items[s], g.d_nitems[s], g.grid[s], 0,
                            g.stream);
        return e;
      };
      hipError_t e = launch_all();
      if (e == hipSuccess) e = hipEventRecord(e0, g.stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_all();
      if (e == hipSuccess) e = hipEventRecord(e1, g.stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        st = hip_fail(e, "batch autotune launch");
        break;
      }
      if (ms / reps / per < best_ms) {
        best_ms = ms / reps / per;
        best = k;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == LBM_OK && best < 0) st = fail(LBM_ENOMEM, "no tile shape fits the batch workspace");
    const lbm_status r = batch_rebuild(b, st == LBM_OK ? best : -1, 0);
    if (st != LBM_OK) return st;
    if (r != LBM_OK) return r;
    if (best_out) *best_out = best;
    return LBM_OK;
  });
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
  return guarded("lbm_batch_destroy", [&]() -> lbm_status {
    if (!b) return LBM_OK;
    const hipError_t e = hipStreamSynchronize(b->eng.stream);
    for (lbm_ctx* c : b->members) c->batch = nullptr;
    b->eng.destroy();
    delete b;
    return e == hipSuccess ? LBM_OK : hip_fail(e, "hipStreamSynchronize");
  });
}

lbm_status lbm_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
  return guarded("lbm_stream_copy", [&]() -> lbm_status {
    if (!dst || !src) return fail(LBM_EINVAL, "NULL buffer");
    if (bytes % 16) return fail(LBM_EINVAL, "bytes must be a multiple of 16");
    SCLBM_HIP(launch_copy(dst, src, bytes, reinterpret_cast<hipStream_t>(hip_stream)));
    return LBM_OK;
  });
}

}  // extern "C"

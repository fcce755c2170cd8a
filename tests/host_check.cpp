// host_check.cpp -- drives the host side of the C-ABI (include/lbm.h) with no
// GPU: argument validation, tile queries and the serving loop on its host-only
// fake executor (admission, budget, bypass, early retirement of unstable
// requests, concurrent submitters, poll, drain, destroy), and the step
// accounting of a batch tick for engines of one, two and three steps per
// launch.  Built with the
// address and undefined-behaviour sanitizers, and separately with the thread
// sanitizer, by tests/test_host_sanitizers.py; it exits non-zero on the first
// unexpected status.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "lbm.h"
#include "sc_device.h"

static int g_fail = 0;

#define EXPECT(cond)                                                              \
  do {                                                                            \
    if (!(cond)) {                                                                \
      std::fprintf(stderr, "host_check: %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond, \
                   lbm_last_error());                                             \
      ++g_fail;                                                                   \
    }                                                                             \
  } while (0)

static lbm_params params(int n, int storage) {
  lbm_params p{};
  p.nx = n;
  p.ny = n;
  p.G = -5.0;
  p.tau = 1.0;
  p.storage = storage;
  p.rho0 = 1.0;
  return p;
}

static lbm_request request(int n, int64_t steps, const double* drops, int nd, double rho_g) {
  lbm_request r{};
  r.params = params(n, LBM_F32);
  r.init.rho_l = 2.0;
  r.init.rho_g = rho_g;
  r.init.width = 2.0;
  r.init.noise_amp = 1e-3;
  r.init.seed = 1;
  r.drops = drops;
  r.n_drops = nd;
  r.steps = steps;
  return r;
}

static void check_validation() {
  size_t pop = 0, work = 0;
  for (int s = 0; s < 4; ++s) {
    lbm_params p = params(100, s);
    EXPECT(lbm_buffer_bytes(&p, &pop, &work) == LBM_OK);
    EXPECT(pop > 0 && work > 0);
    int32_t k = -1;
    EXPECT(lbm_default_tile(&p, &k) == LBM_OK && k >= 0 && k < lbm_tile_count());
  }
  lbm_params bad = params(100, LBM_F32);
  bad.tau = 0.5;
  EXPECT(lbm_buffer_bytes(&bad, &pop, &work) == LBM_EINVAL);
  bad = params(0, LBM_F32);
  EXPECT(lbm_buffer_bytes(&bad, &pop, &work) == LBM_EINVAL);
  bad = params(100, 7);
  EXPECT(lbm_buffer_bytes(&bad, &pop, &work) == LBM_EINVAL);
  EXPECT(lbm_buffer_bytes(nullptr, &pop, &work) == LBM_EINVAL);
  lbm_params p = params(64, LBM_F32);
  lbm_ctx* ctx = nullptr;
  EXPECT(lbm_create(&p, nullptr, nullptr, 0, nullptr, 0, nullptr, &ctx) == LBM_EINVAL);
  EXPECT(ctx == nullptr);
  EXPECT(lbm_step_n(nullptr, 1) == LBM_EINVAL);
  EXPECT(lbm_interface_metrics(nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_interface_metrics_noalloc(nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_destroy(nullptr) == LBM_OK);
  for (int k = 0; k < lbm_tile_count(); ++k) {
    int32_t w, r, t, pf, c, pa, st;
    EXPECT(lbm_tile_describe(k, &w, &r, &t, &pf, &c, &pa, &st) == LBM_OK);
    int32_t rows = 0, items = 0;
    lbm_params q = params(333, LBM_F16_SHIFTED);
    EXPECT(lbm_tile_layout(&q, k, &rows, &items) == LBM_OK && rows > 0 && items > 0);
  }
  EXPECT(lbm_tile_describe(-1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
         LBM_EINVAL);
  EXPECT(lbm_stream_copy(nullptr, nullptr, 16, nullptr) == LBM_EINVAL);
  EXPECT(lbm_version() != nullptr);
}

static void check_server(int policy) {
  lbm_server_opts o{};
  o.policy = policy;
  o.steps_per_tick = 25;
  o.max_slots = 8;
  o.fake_executor = 1;
  o.fake_mlups = 5000.0;
  lbm_server* s = nullptr;
  EXPECT(lbm_server_create(nullptr, size_t(1) << 30, nullptr, &o, &s) == LBM_OK);
  if (!s) return;
  const double drop[3] = {32.0, 32.0, 10.0};
  // a droplet count beyond what the grid's scratch holds is refused before the
  // array (one droplet here) is read
  lbm_request huge = request(64, 10, drop, 2147483647, 0.15);
  uint64_t t = 0;
  EXPECT(lbm_submit(s, &huge, &t) == LBM_EINVAL);
  // larger than the pool
  lbm_request big = request(16384, 10, drop, 1, 0.15);  // 19 GB of buffers, 1 GiB pool
  EXPECT(lbm_submit(s, &big, &t) == LBM_ENOMEM);
  lbm_request bad = request(64, -1, drop, 1, 0.15);
  EXPECT(lbm_submit(s, &bad, &t) == LBM_EINVAL);
  // concurrent submitters, one unstable request each
  std::atomic<int> ok_submits{0};
  std::vector<std::vector<uint64_t>> tickets(4);
  std::vector<std::thread> th;
  for (int w = 0; w < 4; ++w)
    th.emplace_back([&, w] {
      for (int j = 0; j < 12; ++j) {
        lbm_request r = request(48 + 8 * j, 40 + 10 * w, drop, 1, j == 5 ? -0.2 : 0.15);
        uint64_t tk = 0;
        if (lbm_submit(s, &r, &tk) == LBM_OK) {
          tickets[w].push_back(tk);
          ++ok_submits;
        }
      }
    });
  for (auto& x : th) x.join();
  EXPECT(ok_submits.load() == 48);
  EXPECT(lbm_server_drain(s) == LBM_OK);
  int ok = 0, unstable = 0;
  for (auto& v : tickets)
    for (uint64_t tk : v) {
      lbm_result res{};
      const lbm_status st = lbm_poll(s, tk, &res);
      ok += st == LBM_OK;
      unstable += st == LBM_EUNSTABLE;
      EXPECT(res.t_submit <= res.t_admit && res.t_admit <= res.t_done);
      lbm_result again{};
      EXPECT(lbm_poll(s, tk, &again) == LBM_ENOTFOUND);
    }
  EXPECT(ok == 44 && unstable == 4);
  lbm_server_stats st{};
  EXPECT(lbm_server_get_stats(s, &st) == LBM_OK);
  EXPECT(st.completed == 48 && st.unstable == 4 && st.retired_early == 4);
  EXPECT(lbm_server_destroy(s) == LBM_OK);
}

// One tick of a batch engine as its graph orders the launches (the main
// launches, then for three steps per launch the two-step tail, then for two
// or three the single-step tail): for every tick length T, member step count
// nsub <= T and starting buffer, the launches that run advance the member by
// exactly nsub steps, each reads the buffer the one before it wrote, and
// tick_flips counts them.
static void check_tick_accounting() {
  using namespace sclbm;
  for (int K = 1; K <= 3; ++K)
    for (int T = 1; T <= 40; ++T)
      for (int nsub = 0; nsub <= T; ++nsub)
        for (int parity = 0; parity < 2; ++parity) {
          InstDesc d{};
          d.parity = parity;
          d.nsub = nsub;
          d.per_launch = K;
          int steps = 0, flips = 0, buf = parity, misread = 0;
          auto launch = [&](bool runs, int reads, int n) {
            if (!runs) return;
            misread += reads != buf;
            buf ^= 1;
            steps += n;
            ++flips;
          };
          const int main_launches = K == 3 ? T / 3 : (K == 2 ? (T + 1) / 2 : T);
          for (int j = 0; j < main_launches; ++j) {
            if (K == 1) launch(step_runs(&d, j), step_parity(&d, j), 1);
            if (K == 2) launch(pair_runs(&d, j), pair_parity(&d, j), 2);
            if (K == 3) launch(multi_runs(&d, j, 3), pair_parity(&d, j), 3);
          }
          if (K == 3) launch(pair_runs(&d, kTail2Sub), pair_parity(&d, kTail2Sub), 2);
          if (K >= 2) launch(step_runs(&d, kTailSub), step_parity(&d, kTailSub), 1);
          EXPECT(steps == nsub);
          EXPECT(misread == 0);
          EXPECT(flips == tick_flips(nsub, K));
        }
}

int main() {
  check_tick_accounting();
  check_validation();
  check_server(LBM_POLICY_CONTINUOUS);
  check_server(LBM_POLICY_FIFO);
  lbm_server_opts o{};
  o.policy = 9;
  lbm_server* s = nullptr;
  EXPECT(lbm_server_create(nullptr, 1 << 20, nullptr, &o, &s) == LBM_EINVAL);
  if (g_fail) {
    std::fprintf(stderr, "host_check: %d failures\n", g_fail);
    return 1;
  }
  std::printf("host_check: ok\n");
  return 0;
}

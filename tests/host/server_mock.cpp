// Host-only harness for the request server (csrc/server.hpp): the real
// scheduler, admission, HIP gate and memory estimate, over a stand-in handle
// whose setup and CG chunks take random host time instead of GPU work.  Built
// with AddressSanitizer/UBSan and with ThreadSanitizer by
// tests/test_server_host.py; no GPU is touched.
//
// usage: server_mock <geometry file> <max_active> <workers> <cap_factor> <seed> <mode>
//   geometry file: one request per line, "dim n0 n1 n2 tau nsub0 nsub1 nsub2 cuts..."
//   cap_factor:    mem_cap = cap_factor * the largest estimate (0: unlimited)
//   mode 0:        submit every request at random small intervals, poll all, check
//   mode 1:        submit every request, destroy the server at once (drops the queue)
//   mode 2:        keyed requests: every request five times under one key (its own
//                  source each time) beside unkeyed copies, poll all, check outputs,
//                  batches and that resident problems are released at destroy
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <random>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bddc.h"
#include "../../paper_1901_02090_amd/csrc/gate.hpp"
#include "../../paper_1901_02090_amd/csrc/layout.hpp"
#include "../../paper_1901_02090_amd/csrc/nd.hpp"

using namespace bddc;

// ---- stand-ins for the HIP calls the server makes ----------------------------
typedef int hipError_t;
constexpr hipError_t hipSuccess = 0, hipErrorOutOfMemory = 2;
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipMemGetInfo(size_t *fr, size_t *tot) {
  *fr = (size_t)1 << 38;
  *tot = (size_t)1 << 38;
  return hipSuccess;
}
inline const char *hipGetErrorString(hipError_t) { return "stand-in"; }

// ---- what server.hpp takes from the library -------------------------------------
inline int64_t gp_size(int n) {
  const int64_t G = (n + 3) / 4;
  return 8 * G * (G + 1);
}
inline int ld4(int n) { return (n + 3) & ~3; }
inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }
constexpr int TOP_DEFAULT_DOFS = 4096;
constexpr int TOP_BATCH = 128;

using sclock_t = std::chrono::steady_clock;

std::atomic<int> g_live{0};   // stand-in handles alive

// The library's device-memory hook (bddc_set_allocator): the stand-in handle
// takes a few blocks through it at setup and hands them back when destroyed,
// on whichever server thread does that, as the real handle does.
struct Allocator {
  void *(*alloc)(size_t, void *) = nullptr;
  void (*free)(void *, void *) = nullptr;
  void *ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;
std::atomic<long> g_blocks{0};   // blocks taken through the hook and not yet handed back

struct bddc_problem {
  bddc_problem() { ++g_live; }
  ~bddc_problem() {
    for (auto &b : blocks) {
      if (b.second.free) b.second.free(b.first, b.second.ctx);
      else std::free(b.first);
      --g_blocks;
    }
    --g_live;
  }
  std::vector<std::pair<void *, Allocator>> blocks;
  void take(size_t bytes) {
    Allocator a;
    {
      std::lock_guard<std::mutex> lk(g_alloc_mu);
      a = g_alloc;
    }
    void *p = a.alloc ? a.alloc(bytes, a.ctx) : std::malloc(bytes);
    if (!p) throw std::bad_alloc();
    blocks.emplace_back(p, a);
    ++g_blocks;
  }
  Layout L;
  struct Run {
    bool stop = false;
    int chunks = 0, checked = 0;
  } run;
  bddc_stats_t stats{};
  double device_bytes = 0, peak_bytes = 0;
  int ncu = 0;
  // stand-in state
  int target = 1;
  bool block_ready = false;
  double est = 0.0;
  std::vector<sclock_t::time_point> land;
  const double *rhs = nullptr;
  double *flux = nullptr, *pres = nullptr;
  std::mt19937_64 rng;
};

namespace {

thread_local std::string g_last_error;

struct Error {
  int code;
  std::string msg;
};

#define HIPCHK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) throw Error{BDDC_EDEVICE, std::string(#x) + ": stand-in"}; \
  } while (0)

template <typename F>
int guarded(F &&fn) {
  try {
    return fn();
  } catch (const Error &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return BDDC_EDEVICE;
  }
}

double estimate_bytes(const bddc_grid *gr, const bddc_partition *part, double tau, const bddc_options *opt,
                      bool block_vectors);

void sleep_us(double us) { std::this_thread::sleep_for(std::chrono::duration<double, std::micro>(us)); }

// Setup stand-in: the real layout and validation, a random setup time, and a
// footprint below the estimate.  A permeability of 7777 in the first cell
// fails the "factorization".
bddc_problem *make_problem(const bddc_grid *g, const double *perm, const bddc_partition *part, double tau,
                           const bddc_options *opt) {
  GateShared gate(g_gate);
  auto *h = new bddc_problem();
  try {
    int n[3] = {g->n[0], g->n[1], g->n[2]};
    double hh[3] = {g->h[0], g->h[1], g->h[2]};
    const int *cuts[3] = {part->cuts[0], part->cuts[1], part->cuts[2]};
    try {
      h->L.build(g->dim, n, hh, part->nsub, cuts);
    } catch (const std::exception &e) {
      throw Error{BDDC_EINVAL, e.what()};
    }
    for (int64_t c = 0; c < h->L.ncells * h->L.dim; ++c)
      if (!(perm[c] > 0.0)) throw Error{BDDC_EINVAL, "permeability must be finite and > 0"};
    if (perm[0] == 7777.0) throw Error{BDDC_EFACTOR, "stand-in factorization failure"};
    const double est = estimate_bytes(g, part, tau, opt, true);
    h->est = est;
    h->rng.seed((uint64_t)h->L.ncells * 1000003u + (uint64_t)h->L.N);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    h->device_bytes = est * (0.5 + 0.5 * u(h->rng));
    h->peak_bytes = est * (0.8 + 0.2 * u(h->rng));
    h->target = 1 + h->L.N % 4;
    h->ncu = h->L.nF;
    for (int k = 0; k < 3; ++k) h->take(64 + (size_t)(4096 * u(h->rng)));
    sleep_us(3000.0 * u(h->rng));
    h->stats.t_setup_ms = 1.0;
  } catch (...) {
    delete h;
    throw;
  }
  return h;
}

bool solve_needs_cg(const bddc_problem *h) { return h->L.N > 1; }

void solve_begin(bddc_problem *h, const double *rhs, double rtol, double *flux, double *pressure, uint32_t) {
  GateShared g(g_gate);
  if (!(rtol > 0.0)) throw Error{BDDC_EINVAL, "rtol must be > 0"};
  double sum = 0.0, asum = 0.0;
  for (int64_t c = 0; c < h->L.ncells; ++c) {
    sum += rhs[c];
    asum += std::fabs(rhs[c]);
  }
  if (std::fabs(sum) > 1e-12 * asum) throw Error{BDDC_EINVAL, "source must sum to zero"};
  h->run = bddc_problem::Run();
  h->rhs = rhs;
  h->flux = flux;
  h->pres = pressure;
  h->land.clear();
}

void solve_chunk(bddc_problem *h) {
  GateShared g(g_gate);
  auto &R = h->run;
  if (R.chunks - R.checked >= 2) throw Error{BDDC_EINVAL, "at most two CG chunks in flight"};
  std::uniform_real_distribution<double> u(50.0, 500.0);
  h->land.push_back(sclock_t::now() + std::chrono::microseconds((int64_t)u(h->rng)));
  ++R.chunks;
}

int solve_poll(bddc_problem *h, bool wait) {
  GateShared g(g_gate);
  auto &R = h->run;
  if (R.checked >= R.chunks) return 0;
  const auto t = h->land[R.checked];
  if (wait)
    std::this_thread::sleep_until(t);
  else if (sclock_t::now() < t)
    return 0;
  ++R.checked;
  if (R.checked >= h->target) R.stop = true;
  return 1;
}

// Block solve stand-in: every source checked, a random solve time, the same
// outputs per source as solve_finish; the first call "allocates" block vectors.
int block_solve_host(bddc_problem *h, int k, const double *rhs, double rtol, double *flux, double *pressure,
                     int32_t *its, int32_t *conv, double *relres) {
  GateShared g(g_gate);
  if (k <= 0 || k > 16 || !(rtol > 0.0)) throw Error{BDDC_EINVAL, "bad block"};
  const int64_t nc = h->L.ncells, nf = h->L.nfaces_all;
  for (int j = 0; j < k; ++j) {
    double sum = 0.0, asum = 0.0;
    for (int64_t c = 0; c < nc; ++c) {
      sum += rhs[j * nc + c];
      asum += std::fabs(rhs[j * nc + c]);
    }
    if (std::fabs(sum) > 1e-12 * asum) throw Error{BDDC_EINVAL, "source must sum to zero"};
  }
  if (!h->block_ready) {
    h->take(1024);
    h->device_bytes = std::min(h->device_bytes * 1.1, h->est);
    h->block_ready = true;
  }
  std::uniform_real_distribution<double> u(100.0, 1500.0);
  sleep_us(u(h->rng));
  for (int j = 0; j < k; ++j) {
    for (int64_t f = 0; f < nf; ++f) flux[j * nf + f] = (double)f + (double)nc;
    for (int64_t c = 0; c < nc; ++c) pressure[j * nc + c] = 2.0 * rhs[j * nc + c];
    its[j] = 8;
    conv[j] = 1;
    relres[j] = 0.0;
  }
  h->stats.it = 8;
  return BDDC_OK;
}

// Outputs that name the request: flux[j] = j + ncells, pressure = 2 * source.
int solve_finish(bddc_problem *h) {
  auto &R = h->run;
  while (R.checked < R.chunks) solve_poll(h, true);
  GateShared g(g_gate);
  for (int64_t j = 0; j < h->L.nfaces_all; ++j) h->flux[j] = (double)j + (double)h->L.ncells;
  for (int64_t c = 0; c < h->L.ncells; ++c) h->pres[c] = 2.0 * h->rhs[c];
  h->stats.it = 8 * R.chunks;
  h->stats.converged = 1;
  return BDDC_OK;
}

}  // namespace

#include "../../paper_1901_02090_amd/csrc/server.hpp"

extern "C" {
int bddc_set_allocator(void *(*alloc)(size_t, void *), void (*free_fn)(void *, void *), void *ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr)) return BDDC_EINVAL;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = Allocator{alloc, free_fn, ctx};
  return BDDC_OK;
}
long mock_live_handles(void) { return g_live.load(); }
long mock_live_blocks(void) { return g_blocks.load(); }
const char *bddc_last_error(void) { return g_last_error.c_str(); }
}

#ifndef SERVER_MOCK_LIB

struct Req {
  bddc_grid g{};
  std::vector<int32_t> cuts[3];
  double tau = 0.0;
  std::vector<double> perm, rhs;
  bool fail = false;
  uint64_t key = 0;
};

static bool read_requests(const char *path, std::vector<Req> &out) {
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    Req r;
    int nsub[3];
    is >> r.g.dim >> r.g.n[0] >> r.g.n[1] >> r.g.n[2] >> r.tau >> nsub[0] >> nsub[1] >> nsub[2];
    if (!is) return false;
    for (int d = 0; d < 3; ++d) r.g.h[d] = 1.0;
    for (int d = 0; d < r.g.dim; ++d) {
      r.cuts[d].resize(nsub[d] + 1);
      for (auto &c : r.cuts[d]) is >> c;
    }
    const int64_t nc = (int64_t)r.g.n[0] * r.g.n[1] * r.g.n[2];
    r.perm.assign(nc * r.g.dim, 1.0);
    r.rhs.assign(nc, 0.0);
    r.rhs[0] = 1.0;
    r.rhs[nc - 1] = -1.0;
    out.push_back(std::move(r));
  }
  return !out.empty();
}

static bddc_partition part_of(const Req &r) {
  bddc_partition p{};
  for (int d = 0; d < 3; ++d) {
    p.nsub[d] = d < r.g.dim ? (int)r.cuts[d].size() - 1 : 1;
    p.cuts[d] = d < r.g.dim ? r.cuts[d].data() : nullptr;
  }
  return p;
}

int main(int argc, char **argv) {
  if (argc < 7) return 2;
  std::vector<Req> reqs;
  if (!read_requests(argv[1], reqs)) return 3;
  const int max_active = atoi(argv[2]), workers = atoi(argv[3]), mode = atoi(argv[6]);
  const double capf = atof(argv[4]);
  std::mt19937 rng(atoi(argv[5]));
  // every fifth request fails its setup, every seventh has a bad source
  for (size_t k = 0; k < reqs.size(); ++k) {
    if (k % 5 == 3) {
      reqs[k].perm[0] = 7777.0;
      reqs[k].fail = true;
    }
    if (k % 7 == 5 && !reqs[k].fail) {
      reqs[k].rhs[0] += 1.0;
      reqs[k].fail = true;
    }
  }
  if (mode == 2) {
    // every request five times under its own key (the copies get their own
    // sources, failing setups fail the whole key) and once more unkeyed
    std::vector<Req> kr;
    for (size_t k = 0; k < reqs.size(); ++k) {
      for (int c = 0; c < 5; ++c) {
        // (a keyed source must sum to zero at submission: every copy gets a valid one)
        Req q = reqs[k];
        q.key = 1 + k;
        const int64_t nc = (int64_t)q.rhs.size();
        std::fill(q.rhs.begin(), q.rhs.end(), 0.0);
        q.rhs[(c * 7) % nc] += 1.0 + c;
        q.rhs[nc - 1 - (c * 3) % nc] -= 1.0 + c;
        q.fail = q.perm[0] == 7777.0;
        kr.push_back(q);
      }
      kr.push_back(reqs[k]);
    }
    std::shuffle(kr.begin(), kr.end(), rng);
    reqs.swap(kr);
  }
  double est_max = 0.0;
  std::vector<double> est(reqs.size());
  for (size_t k = 0; k < reqs.size(); ++k) {
    const bddc_partition p = part_of(reqs[k]);
    if (bddc_estimate_bytes(&reqs[k].g, &p, reqs[k].tau, nullptr, &est[k]) != BDDC_OK) {
      printf("FAIL estimate %zu: %s\n", k, g_last_error.c_str());
      return 1;
    }
    est_max = std::max(est_max, est[k]);
  }
  bddc_server_options so{};
  so.mem_cap = capf > 0 ? capf * est_max : 0.0;
  so.max_active = max_active;
  so.setup_workers = workers;
  so.precision = BDDC_MIXED;
  bddc_server_handle s = nullptr;
  if (bddc_server_create(&so, &s) != BDDC_OK) return 4;
  std::vector<uint64_t> tick(reqs.size());
  std::uniform_real_distribution<double> gap(0.0, 400.0);
  for (size_t k = 0; k < reqs.size(); ++k) {
    bddc_request rq{};
    rq.grid = reqs[k].g;
    rq.perm = reqs[k].perm.data();
    rq.part = part_of(reqs[k]);
    rq.tau = reqs[k].tau;
    rq.rhs = reqs[k].rhs.data();
    rq.rtol = 1e-8;
    rq.problem_key = reqs[k].key;
    if (bddc_server_submit(s, &rq, &tick[k]) != BDDC_OK) {
      printf("FAIL submit %zu: %s\n", k, g_last_error.c_str());
      return 1;
    }
    if (mode == 0) sleep_us(gap(rng));
  }
  if (mode == 1) {
    bddc_server_destroy(s);
    printf("OK destroyed with %zu requests in flight, %d handles left\n", reqs.size(), g_live.load());
    return 0;
  }
  int bad = 0, busy = 0, failed = 0, batched = 0, reused = 0;
  for (size_t k = 0; k < reqs.size(); ++k) {
    const Req &r = reqs[k];
    const int64_t nc = (int64_t)r.g.n[0] * r.g.n[1] * r.g.n[2];
    int64_t nf = 0;
    for (int d = 0; d < r.g.dim; ++d) {
      int64_t c = 1;
      for (int e = 0; e < 3; ++e) c *= r.g.n[e] + (e == d ? 1 : 0);
      nf += c;
    }
    std::vector<double> flux(nf, -1.0), pres(nc, -1.0);
    bddc_request_stats st{};
    int rc = bddc_server_poll(s, tick[k], 0.0, flux.data(), pres.data(), &st);
    if (rc == BDDC_EBUSY) {
      ++busy;
      rc = bddc_server_poll(s, tick[k], -1.0, flux.data(), pres.data(), &st);
    }
    if (r.fail) {
      if (rc == BDDC_OK) {
        printf("FAIL request %zu should have failed\n", k);
        ++bad;
      }
      ++failed;
      continue;
    }
    if (rc != BDDC_OK || st.status != BDDC_OK) {
      printf("FAIL request %zu: rc %d %s\n", k, rc, g_last_error.c_str());
      ++bad;
      continue;
    }
    for (int64_t j = 0; j < nf; ++j)
      if (flux[j] != (double)j + (double)nc) {
        printf("FAIL request %zu flux %lld\n", k, (long long)j);
        ++bad;
        break;
      }
    for (int64_t c = 0; c < nc; ++c)
      if (pres[c] != 2.0 * r.rhs[c]) {
        printf("FAIL request %zu pressure %lld\n", k, (long long)c);
        ++bad;
        break;
      }
    bddc_options eo{};
    eo.precision = BDDC_MIXED;
    const bddc_partition rp = part_of(r);
    const double e = r.key ? estimate_bytes(&r.g, &rp, r.tau, &eo, true) : est[k];
    if (st.est_bytes != e || st.latency_ms < st.queue_ms || st.batch < 1 || st.batch > 16 ||
        (r.key == 0 && (st.batch != 1 || st.reused))) {
      printf("FAIL request %zu stats\n", k);
      ++bad;
    }
    if (st.batch > 1) ++batched;
    if (st.reused) ++reused;
  }
  bddc_server_stats_t ss{};
  bddc_server_stats(s, &ss);
  if (ss.completed + ss.failed != (int64_t)reqs.size() || ss.failed != failed || ss.queued != 0 || ss.active != 0)
    ++bad;
  if (ss.peak_active > max_active) ++bad;
  if (capf > 0 && ss.peak_bytes > so.mem_cap) ++bad;
  if (mode == 2 && reused == 0) ++bad;
  bddc_server_destroy(s);
  if (g_live.load() != 0) ++bad;
  printf("%s requests %zu failed %d busy-at-first-poll %d batched %d reused %d peak_active %d peak %.3g of cap %.3g, "
         "p50 %.2f ms p99 %.2f ms\n",
         bad ? "FAIL" : "OK", reqs.size(), failed, busy, batched, reused, ss.peak_active, ss.peak_bytes, ss.mem_cap,
         ss.p50_ms, ss.p99_ms);
  return bad ? 1 : 0;
}
#endif  // SERVER_MOCK_LIB

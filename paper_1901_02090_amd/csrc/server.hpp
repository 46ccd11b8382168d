// Request loop over independent problems with continuous batching (the
// serving half of the C ABI), and the device-memory estimate it admits by.
//
// Threads:
//   setup workers  take admitted requests in order, build the handle (setup:
//                  factorizations, face eigenproblems, coarse factor) and
//                  enqueue the start of its solve, on the handle's own streams;
//   driver         keeps up to two captured chunks of CG iterations in flight
//                  for every solving request, reads each chunk's state when it
//                  lands (event queries, no blocking), finishes converged
//                  requests, destroys their handles and admits the next ones;
//                  it also releases the idle resident problems that admission
//                  evicted.
// Requests with a problem key share one resident problem: the first sets it
// up (a setup worker), and from then on the waiting requests of the key are
// solved in blocks of up to 16 by a worker (bddc_solve_block's kernels), one
// block after another, while the problem stays resident.
// Requests of different sizes therefore overlap on the device: the kernels of
// several CG chunks and of a setup run at once on different streams.  A
// handle is touched by one thread at a time (its worker, then the driver).
// All bookkeeping sits under one mutex; no HIP call is made while holding it.
// Graph captures (one per handle, by its worker) are kept apart from every
// other thread's HIP calls by the library's HIP gate.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace {

constexpr int EST_ADAPTIVE_ROWS = 8;   // assumed adaptive rows per face before the eigenproblems
constexpr int SERVE_DEPTH = 2;         // CG chunks in flight per solving request

Layout build_layout(const bddc_grid *gr, const bddc_partition *part) {
  if (!gr || !part) throw Error{BDDC_EINVAL, "null argument"};
  if (gr->dim != 2 && gr->dim != 3) throw Error{BDDC_EINVAL, "dim must be 2 or 3"};
  int n[3] = {gr->n[0], gr->n[1], gr->n[2]};
  double hh[3] = {gr->h[0], gr->h[1], gr->h[2]};
  const int *cuts[3] = {part->cuts[0], part->cuts[1], part->cuts[2]};
  for (int d = 0; d < gr->dim; ++d)
    if (!cuts[d]) throw Error{BDDC_EINVAL, "partition cuts missing"};
  Layout L;
  try {
    L.build(gr->dim, n, hh, part->nsub, cuts);
  } catch (const std::exception &e) {
    throw Error{BDDC_EINVAL, e.what()};
  }
  return L;
}

// Sum of the device arrays do_setup and the solve allocate, all taken as held
// at once (the setup workspaces released along the way included); with
// block_vectors, also those of the block CG (16 columns of every CG vector,
// at most 10,000 iterations of coefficient history).
constexpr int SRV_BLOCK = 16;

double estimate_bytes(const bddc_grid *gr, const bddc_partition *part, double tau, const bddc_options *opt,
                      bool block_vectors) {
  const Layout L = build_layout(gr, part);
  const int N = L.N, nF = L.nF, dim = L.dim;
  const bool allc = opt && (opt->flags & BDDC_ALL_CONSTRAINED);
  const bool ms = !allc && opt && (opt->flags & BDDC_MULTISCALE);
  const bool adaptive = !ms && tau > 0.0 && std::isfinite(tau);
  std::vector<int> fk(nF, 0);
  for (int f = 0; f < nF; ++f) {
    const int room = std::max(0, L.f_n[f] - 1);
    fk[f] = allc ? room : ms ? std::min(room, 1) : (adaptive ? std::min(room, EST_ADAPTIVE_ROWS) : 0);
  }
  const double totG = (double)L.g_off[N];
  double b = 0.0;
  // index data, permeability, cell coefficients
  b += 4.0 * ((double)L.ncells + 6.0 * totG + 6.0 * L.nGamma + 8.0 * nF + 16.0 * N +
              (double)L.sub_faces.size() + (double)L.line_g.size());
  b += 8.0 * ((double)L.ncells * (dim + 3) + 2.0 * N + (double)L.line_off.size());
  // local setup workspaces, extension operators X^i, packed S^i
  for (int i = 0; i < N; ++i) {
    const double nc = L.nc[i], nG = L.nG[i];
    b += 8.0 * (2 * nc * nc + nc * (nG + 1) + 3 * nG * nG) + 8.0 * nc * nc + 8.0 * (double)gp_size(L.nG[i]) + 64.0;
  }
  // face eigenproblems
  for (int f = 0; f < nF; ++f) {
    const double fn = L.f_n[f];
    b += 8.0 * fn * fn;
    if (adaptive || allc || ms) b += 8.0 * (6 * fn * fn + fn) + 8.0 * fn + 40.0;
  }
  // local coarse spaces: workspaces, A_c^i, Psi^i (FP64 + FP32), T^i (FP64 + FP32)
  double sum_nci = 0.0;
  for (int i = 0; i < N; ++i) {
    double nci = 0.0;
    for (int t = L.sub_face_off[i]; t < L.sub_face_off[i + 1]; ++t) nci += 1 + fk[L.sub_faces[t]];
    sum_nci += nci;
    const double nG = L.nG[i];
    b += 8.0 * (4 * nci * nG + 2 * nci * nci) + 8.0 * nci * nci + 12.0 * ld4(L.nG[i]) * nci +
         12.0 * (double)gp_size(L.nG[i]) + 32.0;
  }
  // coarse factorization, sweeps and dense top block, on the plan of these counts
  if (N > 1) {
    NdPlan P;
    try {
      nd_plan(L, fk, opt ? opt->coarse_leaf : 0, P);
    } catch (const std::logic_error &e) {
      throw Error{BDDC_EINVAL, std::string("coarse plan: ") + e.what()};
    }
    const int ct = opt ? opt->coarse_top : 0;
    nd_dense_top(P, ct == 0 ? TOP_DEFAULT_DOFS : ct);
    const int nfr = P.nfr;
    const double nk = P.nk, nv = (double)P.v_off[nfr], nb = (double)P.b_off[nfr];
    b += 8.0 * ((double)P.F_off[nfr] + (double)P.w_off[nfr] + (double)P.q_off[nfr] + 2.0 * (double)P.r_off[nfr]);
    b += 8.0 * (5 * nk + 2 * nv + nb) + 4.0 * ((double)P.task.size() + 2 * nb + 16.0 * nfr + 2 * nk);
    if (P.nt > 0) {
      const double ld = (P.nt + 1) & ~1, cols = std::min(P.nt, TOP_BATCH);
      b += 8.0 * P.nt * ld + 8.0 * cols * (3 * nk + 2 * nv + std::max(nb, 1.0)) + 4.0 * (double)P.tg.size();
    }
    if (block_vectors)
      b += 8.0 * SRV_BLOCK * (3 * nk + 2 * nv + nb + P.nt) + 4.0 * 12.0 * 2.0 * (nv / 64.0 + 2.0 * nfr);
  }
  if (block_vectors) {
    const int maxit = opt && opt->max_it > 0 ? opt->max_it : 10000;
    b += 8.0 * SRV_BLOCK * (6.0 * L.nGamma + 2.0 * totG + 2.0 * N + 3.0 * 512 + 2.0 * (maxit + 2)) + 4096.0;
  }
  // CG and output vectors
  b += 8.0 * (7.0 * L.nGamma + 2.0 * N + 2.0 * totG + sum_nci + 6.0 * (double)L.ncells + (double)L.nfaces_all +
              2.0 * nblk(L.nGamma) + nF + 1024 + 20000.0);
  return b;
}

using sclock = std::chrono::steady_clock;

double ms_between(sclock::time_point a, sclock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

namespace bddc {

struct Resident;

struct SrvRequest {
  uint64_t id = 0;
  bddc_grid grid{};
  int32_t nsub[3] = {1, 1, 1};
  std::vector<int32_t> cuts[3];
  std::vector<double> perm, rhs, flux, pres;
  double tau = 0.0, rtol = 1e-8;
  int32_t max_it = 0;
  double est = 0.0, held = 0.0;   // admission estimate; bytes counted against the cap now
  enum State { QUEUED, SETUP, SOLVING, DONE } state = QUEUED;
  bddc_problem *h = nullptr;
  Resident *res = nullptr;        // keyed: the shared problem
  bool reused = false;            // keyed and not the one that set it up
  int status = BDDC_OK;
  std::string err;
  bddc_request_stats st{};
  sclock::time_point t_submit, t_admit, t_setup_end, t_done;

  bddc_partition partition() const {
    bddc_partition p{};
    for (int d = 0; d < 3; ++d) {
      p.nsub[d] = nsub[d];
      p.cuts[d] = cuts[d].empty() ? nullptr : cuts[d].data();
    }
    return p;
  }
};

// A problem shared by the requests of one key: set up once, resident until
// evicted or the server is destroyed.  busy: a worker owns it (setting it up
// or solving blocks); ready: set up.
struct Resident {
  uint64_t key = 0;
  bddc_grid grid{};
  int32_t nsub[3] = {1, 1, 1};
  std::vector<int32_t> cuts[3];
  double tau = 0.0;
  bddc_problem *h = nullptr;
  bool ready = false, busy = true;
  double held = 0.0;                   // bytes counted against the cap once set up
  std::deque<SrvRequest *> pending;    // waiting to be solved
  sclock::time_point last_use;
};

}  // namespace bddc

struct bddc_server {
  bddc_server_options opt{};
  double cap = 0.0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_setup, cv_drive, cv_done;
  std::deque<SrvRequest *> queue;      // waiting for admission, in arrival order
  std::deque<SrvRequest *> to_setup;   // admitted, waiting for a worker
  std::vector<SrvRequest *> ready;     // set up, handed to the driver
  std::unordered_map<uint64_t, std::unique_ptr<SrvRequest>> reqs;
  std::unordered_map<uint64_t, std::unique_ptr<Resident>> residents;   // by problem key
  std::deque<Resident *> batch_jobs;   // ready residents with waiting requests, no worker on them
  std::vector<std::unique_ptr<Resident>> evicted;   // released by the driver (outside the lock)
  uint64_t next_id = 1;
  double committed = 0.0, peak_committed = 0.0;
  int admitted = 0, peak_admitted = 0, in_setup = 0;
  bool stopping = false;
  int64_t n_submitted = 0, n_completed = 0, n_failed = 0;
  std::vector<double> lat_ms;
  bool any_submit = false;
  sclock::time_point t_first, t_last;
  std::thread driver;
  std::vector<std::thread> workers;

  // Under mu: admit from the head of the queue while a slot is free and the
  // estimate fits next to what is held; when it does not fit, the idle
  // resident problem used longest ago is evicted (the driver frees it).
  void admit_locked() {
    while (!queue.empty() && admitted < opt.max_active) {
      SrvRequest *r = queue.front();
      if (committed + r->est > cap) {
        Resident *lru = nullptr;
        for (auto &kv : residents) {
          Resident *q = kv.second.get();
          if (q->ready && !q->busy && q->pending.empty() && (!lru || q->last_use < lru->last_use)) lru = q;
        }
        if (lru) {
          auto it = residents.find(lru->key);
          evicted.push_back(std::move(it->second));
          residents.erase(it);
          cv_drive.notify_one();
        }
        break;
      }
      queue.pop_front();
      r->t_admit = sclock::now();
      r->held = r->est;
      committed += r->est;
      peak_committed = std::max(peak_committed, committed);
      ++admitted;
      peak_admitted = std::max(peak_admitted, admitted);
      to_setup.push_back(r);
      cv_setup.notify_one();
    }
  }

  // Under mu: a request leaves (done or failed); its bytes and slot free up.
  void retire_locked(SrvRequest *r) {
    committed -= r->held;
    r->held = 0.0;
    --admitted;
    complete_locked(r);
    admit_locked();
  }

  // Under mu: a request is done (its statistics, the latency record).
  void complete_locked(SrvRequest *r) {
    r->state = SrvRequest::DONE;
    r->t_done = sclock::now();
    r->st.status = r->status;
    r->st.queue_ms = ms_between(r->t_submit, r->t_admit);
    r->st.latency_ms = ms_between(r->t_submit, r->t_done);
    r->st.solve_ms = ms_between(r->t_setup_end, r->t_done);
    if (r->status == BDDC_OK || r->status == BDDC_ENOCONV) {
      ++n_completed;
      lat_ms.push_back(r->st.latency_ms);
      t_last = r->t_done;
    } else {
      ++n_failed;
    }
    cv_done.notify_all();
  }

  void fail(SrvRequest *r, int code, const std::string &msg) {
    r->status = code;
    r->err = msg;
  }

  void worker_loop() {
    (void)hipSetDevice(device);
    for (;;) {
      SrvRequest *r = nullptr;
      Resident *job = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_setup.wait(lk, [&] { return stopping || !to_setup.empty() || !batch_jobs.empty(); });
        if (!batch_jobs.empty()) {
          job = batch_jobs.front();
          batch_jobs.pop_front();
        } else if (!to_setup.empty()) {
          r = to_setup.front();
          to_setup.pop_front();
          r->state = SrvRequest::SETUP;
          ++in_setup;
        } else {
          return;
        }
      }
      if (job) {
        run_batches(job);
        continue;
      }
      if (r->res) {
        setup_resident(r);
        continue;
      }
      bool ok = false;
      try {
        bddc_options o{};
        o.precision = opt.precision;
        o.max_it = r->max_it;
        o.flags = opt.flags;
        const bddc_partition part = r->partition();
        r->h = make_problem(&r->grid, r->perm.data(), &part, r->tau, &o);
        r->flux.assign(r->h->L.nfaces_all, 0.0);
        r->pres.assign(r->h->L.ncells, 0.0);
        solve_begin(r->h, r->rhs.data(), r->rtol, r->flux.data(), r->pres.data(), 0);
        r->st.setup_ms = r->h->stats.t_setup_ms;
        r->st.peak_bytes = r->h->peak_bytes;
        r->st.device_bytes = r->h->device_bytes;
        ok = true;
      } catch (const Error &e) {
        fail(r, e.code, e.msg);
      } catch (const std::bad_alloc &) {
        fail(r, BDDC_ENOMEM, "host out of memory");
      } catch (const std::exception &e) {
        fail(r, BDDC_EDEVICE, e.what());
      }
      r->t_setup_end = sclock::now();
      r->perm.clear();
      r->perm.shrink_to_fit();
      bddc_problem *dead = nullptr;
      {
        std::lock_guard<std::mutex> lk(mu);
        --in_setup;
        if (ok) {
          // the setup peak has passed: count what the handle holds now
          committed += r->h->device_bytes - r->held;
          r->held = r->h->device_bytes;
          peak_committed = std::max(peak_committed, committed);
          r->state = SrvRequest::SOLVING;
          ready.push_back(r);
          cv_drive.notify_one();
        } else {
          dead = r->h;
          r->h = nullptr;
          retire_locked(r);
        }
        admit_locked();
      }
      if (dead) {
        GateShared g(g_gate);
        delete dead;
      }
    }
  }

  // The first request of a key: set the shared problem up, then solve the
  // waiting requests of the key (this one included) in blocks.
  void setup_resident(SrvRequest *r) {
    Resident *res = r->res;
    bddc_problem *h = nullptr;
    try {
      bddc_options o{};
      o.precision = opt.precision;
      o.max_it = r->max_it;
      o.flags = opt.flags;
      const bddc_partition part = r->partition();
      h = make_problem(&r->grid, r->perm.data(), &part, r->tau, &o);
      r->st.setup_ms = h->stats.t_setup_ms;
      r->st.peak_bytes = h->peak_bytes;
    } catch (const Error &e) {
      fail(r, e.code, e.msg);
    } catch (const std::bad_alloc &) {
      fail(r, BDDC_ENOMEM, "host out of memory");
    } catch (const std::exception &e) {
      fail(r, BDDC_EDEVICE, e.what());
    }
    r->t_setup_end = sclock::now();
    r->perm.clear();
    r->perm.shrink_to_fit();
    {
      std::lock_guard<std::mutex> lk(mu);
      --in_setup;
      if (h) {
        // the problem's bytes move from the request to the resident problem,
        // and the request's slot frees up
        // (it keeps the estimate, which holds the block vectors of its first block solve)
        res->h = h;
        res->held = std::max(r->held, h->device_bytes);
        committed += res->held - r->held;
        peak_committed = std::max(peak_committed, committed);
        r->held = 0.0;
        --admitted;
        res->ready = true;
        admit_locked();
      } else {
        // every request of the key fails with the setup
        for (SrvRequest *q : res->pending)
          if (q != r) {
            q->status = r->status;
            q->err = r->err;
            complete_locked(q);
          }
        res->pending.clear();
        r->res = nullptr;
        residents.erase(res->key);
        retire_locked(r);
        return;
      }
    }
    run_batches(res);
  }

  // Solve the waiting requests of a ready resident problem in blocks of up to
  // 16 with equal rtol, until none is left; then the problem is idle.
  void run_batches(Resident *res) {
    bddc_problem *h = res->h;
    const int64_t nc = h->L.ncells, nf = h->L.nfaces_all;
    for (;;) {
      std::vector<SrvRequest *> b;
      double rtol = 0.0;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (res->pending.empty()) {
          res->busy = false;
          res->last_use = sclock::now();
          admit_locked();
          return;
        }
        rtol = res->pending.front()->rtol;
        for (auto it = res->pending.begin(); it != res->pending.end() && (int)b.size() < 16;) {
          if ((*it)->rtol == rtol) {
            b.push_back(*it);
            it = res->pending.erase(it);
          } else {
            ++it;
          }
        }
        for (SrvRequest *q : b) q->state = SrvRequest::SOLVING;
      }
      const int k = (int)b.size();
      std::vector<double> rhs((size_t)k * nc), fl((size_t)k * nf, 0.0), pr((size_t)k * nc, 0.0), rel(k, 0.0);
      std::vector<int32_t> its(k, 0), conv(k, 0);
      for (int j = 0; j < k; ++j) std::copy(b[j]->rhs.begin(), b[j]->rhs.end(), rhs.begin() + (size_t)j * nc);
      int rc = BDDC_OK;
      std::string err;
      try {
        rc = block_solve_host(h, k, rhs.data(), rtol, fl.data(), pr.data(), its.data(), conv.data(), rel.data());
        if (rc != BDDC_OK) err = rc == BDDC_ENOCONV ? "maximum number of CG iterations reached" : "CG breakdown";
      } catch (const Error &e) {
        rc = e.code;
        err = e.msg;
      } catch (const std::exception &e) {
        rc = BDDC_EDEVICE;
        err = e.what();
      }
      std::lock_guard<std::mutex> lk(mu);
      // the first block solve allocates the block vectors (counted in the estimate)
      if (h->device_bytes > res->held) {
        committed += h->device_bytes - res->held;
        res->held = h->device_bytes;
        peak_committed = std::max(peak_committed, committed);
      }
      const bool solved = rc == BDDC_OK || rc == BDDC_ENOCONV || rc == BDDC_EBREAKDOWN;
      for (int j = 0; j < k; ++j) {
        SrvRequest *q = b[j];
        if (solved) {
          q->flux.assign(fl.begin() + (size_t)j * nf, fl.begin() + (size_t)(j + 1) * nf);
          q->pres.assign(pr.begin() + (size_t)j * nc, pr.begin() + (size_t)(j + 1) * nc);
          q->status = conv[j] ? BDDC_OK : (rc == BDDC_EBREAKDOWN ? BDDC_EBREAKDOWN : BDDC_ENOCONV);
          if (q->status != BDDC_OK) q->err = err;
        } else {
          q->status = rc;
          q->err = err;
        }
        q->st.it = its[j];
        q->st.converged = conv[j];
        q->st.relres = rel[j];
        q->st.kappa = j == k - 1 ? h->stats.kappa : 0.0;
        q->st.n_sub = h->L.N;
        q->st.n_coarse = h->ncu + h->L.N;
        q->st.est_bytes = q->est;
        q->st.device_bytes = res->held;
        q->st.batch = k;
        q->st.reused = q->reused ? 1 : 0;
        complete_locked(q);
      }
    }
  }

  // Advance one solving request without blocking on the device; true when it
  // has left (finished or failed).
  bool advance(SrvRequest *r, bool &progressed) {
    bddc_problem *h = r->h;
    auto &R = h->run;
    int rc = BDDC_OK;
    try {
      if (solve_needs_cg(h)) {
        while (!R.stop && R.chunks - R.checked < SERVE_DEPTH) {
          solve_chunk(h);
          progressed = true;
        }
        if (solve_poll(h, false)) progressed = true;
        if (!R.stop) return false;
      }
      rc = solve_finish(h);
      r->status = rc;
      if (rc == BDDC_ENOCONV) r->err = "maximum number of CG iterations reached";
    } catch (const Error &e) {
      fail(r, e.code, e.msg);
    } catch (const std::exception &e) {
      fail(r, BDDC_EDEVICE, e.what());
    }
    progressed = true;
    r->st.it = h->stats.it;
    r->st.converged = h->stats.converged;
    r->st.relres = h->stats.relres;
    r->st.kappa = h->stats.kappa;
    r->st.n_sub = h->L.N;
    r->st.n_coarse = h->ncu + h->L.N;
    r->st.est_bytes = r->est;
    r->st.batch = 1;
    r->h = nullptr;
    {
      GateShared g(g_gate);
      delete h;
    }
    std::lock_guard<std::mutex> lk(mu);
    retire_locked(r);
    return true;
  }

  // Free the handles of the evicted resident problems (HIP calls outside the
  // lock), then count their bytes as free.
  void release_evicted() {
    std::vector<std::unique_ptr<Resident>> ev;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (evicted.empty()) return;
      ev.swap(evicted);
    }
    double freed = 0.0;
    for (auto &q : ev) {
      freed += q->held;
      GateShared g(g_gate);
      delete q->h;
      q->h = nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    committed -= freed;
    admit_locked();
  }

  void driver_loop() {
    (void)hipSetDevice(device);
    std::vector<SrvRequest *> act;
    for (;;) {
      release_evicted();
      {
        std::unique_lock<std::mutex> lk(mu);
        act.insert(act.end(), ready.begin(), ready.end());
        ready.clear();
        if (act.empty()) {
          if (stopping && to_setup.empty() && in_setup == 0 && evicted.empty()) return;
          cv_drive.wait_for(lk, std::chrono::milliseconds(2));
          continue;
        }
      }
      bool progressed = false;
      for (size_t k = 0; k < act.size();) {
        if (advance(act[k], progressed)) {
          act[k] = act.back();
          act.pop_back();
        } else {
          ++k;
        }
      }
      if (!progressed) {
        std::unique_lock<std::mutex> lk(mu);
        cv_drive.wait_for(lk, std::chrono::microseconds(20), [&] { return !ready.empty(); });
      }
    }
  }
};

extern "C" {

int bddc_estimate_bytes(const bddc_grid *g, const bddc_partition *part, double tau, const bddc_options *opt,
                        double *bytes) {
  return guarded([&]() -> int {
    if (!bytes) throw Error{BDDC_EINVAL, "null argument"};
    *bytes = estimate_bytes(g, part, tau, opt, false);
    return BDDC_OK;
  });
}

int bddc_server_create(const bddc_server_options *opt, bddc_server_handle *out) {
  return guarded([&]() -> int {
    if (!out) throw Error{BDDC_EINVAL, "null argument"};
    *out = nullptr;
    auto sv = std::make_unique<bddc_server>();
    if (opt) sv->opt = *opt;
    if (sv->opt.max_active <= 0) sv->opt.max_active = 4;
    if (sv->opt.setup_workers <= 0) sv->opt.setup_workers = 1;
    if (sv->opt.precision != BDDC_FP64 && sv->opt.precision != BDDC_MIXED) throw Error{BDDC_EINVAL, "bad precision"};
    HIPCHK(hipGetDevice(&sv->device));
    sv->cap = sv->opt.mem_cap;
    if (!(sv->cap > 0.0)) {
      size_t fr = 0, tot = 0;
      HIPCHK(hipMemGetInfo(&fr, &tot));
      sv->cap = 0.9 * (double)fr;
    }
    bddc_server *s = sv.get();
    s->driver = std::thread([s] { s->driver_loop(); });
    for (int k = 0; k < s->opt.setup_workers; ++k) s->workers.emplace_back([s] { s->worker_loop(); });
    *out = sv.release();
    return BDDC_OK;
  });
}

int bddc_server_submit(bddc_server_handle s, const bddc_request *req, uint64_t *ticket) {
  return guarded([&]() -> int {
    if (!s || !req || !ticket || !req->perm || !req->rhs) throw Error{BDDC_EINVAL, "null argument"};
    if (!(req->rtol > 0.0)) throw Error{BDDC_EINVAL, "rtol must be > 0"};
    auto r = std::make_unique<SrvRequest>();
    bddc_options o{};
    o.precision = s->opt.precision;
    o.flags = s->opt.flags;
    // validates grid and partition; a keyed problem's estimate holds its block vectors too
    r->est = estimate_bytes(&req->grid, &req->part, req->tau, &o, req->problem_key != 0);
    if (r->est > s->cap) throw Error{BDDC_ENOMEM, "request estimate exceeds the server's memory cap"};
    const Layout L = build_layout(&req->grid, &req->part);
    r->grid = req->grid;
    for (int d = 0; d < 3; ++d) {
      r->nsub[d] = req->part.nsub[d];
      if (d < req->grid.dim) r->cuts[d].assign(req->part.cuts[d], req->part.cuts[d] + req->part.nsub[d] + 1);
    }
    r->perm.assign(req->perm, req->perm + L.ncells * L.dim);
    r->rhs.assign(req->rhs, req->rhs + L.ncells);
    r->tau = req->tau;
    r->rtol = req->rtol;
    r->max_it = req->max_it;
    r->t_submit = sclock::now();
    const uint64_t key = req->problem_key;
    if (key) {
      // a keyed request is solved in a block with others: its source is
      // checked here, so that a bad one fails alone
      double sum = 0.0, asum = 0.0;
      for (double v : r->rhs) {
        if (!std::isfinite(v)) throw Error{BDDC_EINVAL, "source must be finite"};
        sum += v;
        asum += std::fabs(v);
      }
      if (std::fabs(sum) > 1e-12 * asum) throw Error{BDDC_EINVAL, "source must sum to zero (no-flow compatibility)"};
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) throw Error{BDDC_EINVAL, "server is shutting down"};
    Resident *res = nullptr;
    if (key) {
      auto it = s->residents.find(key);
      if (it != s->residents.end()) {
        res = it->second.get();
        bool same = res->grid.dim == r->grid.dim && res->tau == r->tau;
        for (int d = 0; d < 3 && same; ++d)
          same = res->grid.n[d] == r->grid.n[d] && res->grid.h[d] == r->grid.h[d] && res->nsub[d] == r->nsub[d] &&
                 res->cuts[d] == r->cuts[d];
        if (!same) throw Error{BDDC_EINVAL, "request differs from the resident problem of its key"};
      }
    }
    SrvRequest *rp = r.get();
    rp->id = s->next_id++;
    *ticket = rp->id;
    if (!s->any_submit) {
      s->any_submit = true;
      s->t_first = rp->t_submit;
    }
    ++s->n_submitted;
    s->reqs[rp->id] = std::move(r);
    if (res) {
      // the problem is resident (or being set up): wait for the next block
      rp->res = res;
      rp->reused = true;
      rp->t_admit = rp->t_setup_end = rp->t_submit;
      rp->perm.clear();
      rp->perm.shrink_to_fit();
      res->pending.push_back(rp);
      if (res->ready && !res->busy) {
        res->busy = true;
        s->batch_jobs.push_back(res);
        s->cv_setup.notify_one();
      }
    } else {
      if (key) {
        auto nr = std::make_unique<Resident>();
        nr->key = key;
        nr->grid = rp->grid;
        nr->tau = rp->tau;
        for (int d = 0; d < 3; ++d) {
          nr->nsub[d] = rp->nsub[d];
          nr->cuts[d] = rp->cuts[d];
        }
        rp->res = nr.get();
        nr->pending.push_back(rp);
        s->residents[key] = std::move(nr);
      }
      s->queue.push_back(rp);
    }
    s->admit_locked();
    return BDDC_OK;
  });
}

int bddc_server_poll(bddc_server_handle s, uint64_t ticket, double wait_ms, double *flux, double *pressure,
                     bddc_request_stats *st) {
  return guarded([&]() -> int {
    if (!s) throw Error{BDDC_EINVAL, "null argument"};
    std::unique_ptr<SrvRequest> r;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      auto it = s->reqs.find(ticket);
      if (it == s->reqs.end()) throw Error{BDDC_EINVAL, "unknown ticket"};
      SrvRequest *q = it->second.get();
      auto done = [&] { return q->state == SrvRequest::DONE; };
      if (wait_ms < 0)
        s->cv_done.wait(lk, done);
      else if (wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(wait_ms), done);
      if (!done()) return BDDC_EBUSY;
      r = std::move(it->second);
      s->reqs.erase(it);
    }
    if (flux && !r->flux.empty()) std::copy(r->flux.begin(), r->flux.end(), flux);
    if (pressure && !r->pres.empty()) std::copy(r->pres.begin(), r->pres.end(), pressure);
    if (st) *st = r->st;
    if (r->status != BDDC_OK) g_last_error = r->err;
    return r->status;
  });
}

int bddc_server_stats(bddc_server_handle s, bddc_server_stats_t *out) {
  return guarded([&]() -> int {
    if (!s || !out) throw Error{BDDC_EINVAL, "null argument"};
    std::lock_guard<std::mutex> lk(s->mu);
    bddc_server_stats_t o{};
    o.submitted = s->n_submitted;
    o.completed = s->n_completed;
    o.failed = s->n_failed;
    o.queued = (int64_t)s->queue.size();
    o.active = s->admitted;
    o.peak_active = s->peak_admitted;
    o.peak_bytes = s->peak_committed;
    o.mem_cap = s->cap;
    if (!s->lat_ms.empty()) {
      std::vector<double> v = s->lat_ms;
      std::sort(v.begin(), v.end());
      auto pct = [&](double q) {
        const double x = q * (double)(v.size() - 1);
        const size_t i = (size_t)x;
        const double f = x - (double)i;
        return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
      };
      o.p50_ms = pct(0.50);
      o.p99_ms = pct(0.99);
      const double span = ms_between(s->t_first, s->t_last) * 1e-3;
      o.solves_per_s = span > 0.0 ? (double)s->n_completed / span : 0.0;
    }
    *out = o;
    return BDDC_OK;
  });
}

int bddc_server_destroy(bddc_server_handle s) {
  return guarded([&]() -> int {
    if (!s) return BDDC_OK;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stopping = true;
      for (SrvRequest *r : s->queue) {
        r->status = BDDC_EINVAL;
        r->err = "server destroyed before admission";
        r->state = SrvRequest::DONE;
        if (r->res) {
          // the key's problem will not be set up: its waiting requests go too
          for (SrvRequest *q : r->res->pending)
            if (q != r) {
              q->status = BDDC_EINVAL;
              q->err = "server destroyed before admission";
              q->state = SrvRequest::DONE;
            }
          s->residents.erase(r->res->key);
          r->res = nullptr;
        }
      }
      s->queue.clear();
      s->cv_setup.notify_all();
      s->cv_drive.notify_all();
      s->cv_done.notify_all();
    }
    for (auto &t : s->workers) t.join();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->cv_drive.notify_all();
    }
    s->driver.join();
    for (auto &kv : s->residents) {
      GateShared g(g_gate);
      delete kv.second->h;
      kv.second->h = nullptr;
    }
    delete s;
    return BDDC_OK;
  });
}

}  // extern "C"

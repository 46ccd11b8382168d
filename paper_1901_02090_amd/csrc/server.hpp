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
//                  requests, destroys their handles and admits the next ones.
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
// at once (the setup workspaces released along the way included).
double estimate_bytes(const bddc_grid *gr, const bddc_partition *part, double tau, const bddc_options *opt) {
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
  // estimate fits next to what is held.
  void admit_locked() {
    while (!queue.empty() && admitted < opt.max_active) {
      SrvRequest *r = queue.front();
      if (committed + r->est > cap) break;
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
    admit_locked();
  }

  void fail(SrvRequest *r, int code, const std::string &msg) {
    r->status = code;
    r->err = msg;
  }

  void worker_loop() {
    (void)hipSetDevice(device);
    for (;;) {
      SrvRequest *r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_setup.wait(lk, [&] { return stopping || !to_setup.empty(); });
        if (to_setup.empty()) return;
        r = to_setup.front();
        to_setup.pop_front();
        r->state = SrvRequest::SETUP;
        ++in_setup;
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
    r->h = nullptr;
    {
      GateShared g(g_gate);
      delete h;
    }
    std::lock_guard<std::mutex> lk(mu);
    retire_locked(r);
    return true;
  }

  void driver_loop() {
    (void)hipSetDevice(device);
    std::vector<SrvRequest *> act;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu);
        act.insert(act.end(), ready.begin(), ready.end());
        ready.clear();
        if (act.empty()) {
          if (stopping && to_setup.empty() && in_setup == 0) return;
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
    *bytes = estimate_bytes(g, part, tau, opt);
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
    r->est = estimate_bytes(&req->grid, &req->part, req->tau, &o);   // validates grid and partition
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
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) throw Error{BDDC_EINVAL, "server is shutting down"};
    r->id = s->next_id++;
    *ticket = r->id;
    if (!s->any_submit) {
      s->any_submit = true;
      s->t_first = r->t_submit;
    }
    ++s->n_submitted;
    s->queue.push_back(r.get());
    s->reqs[r->id] = std::move(r);
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
    delete s;
    return BDDC_OK;
  });
}

}  // extern "C"

// Serving: continuous batching of trajectory jobs with HBM-budget admission.
//
// Jobs (one sv_job each) are admitted in arrival order while the device bytes
// they will hold fit in the budget.  Admitted jobs of distance <= 4 join the
// lane of their (d, gate set, dtype, zeta); a worker per lane repeatedly takes
// the trajectories waiting in its lane -- from any number of jobs, oldest
// first -- and runs them in one persistent batched launch on its own stream,
// so a job that arrives while a launch is running joins the next one.  Jobs of
// distance 5 run on one of `big_streams` workers, each with its own stream,
// and overlap on the device with each other and with the lanes.  Every
// trajectory draws from (seed, trajectory index, draw index) only, so a job's
// records do not depend on what it was batched with.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

namespace {

size_t rounds_footprint(int d, int dtype, int n_traj, int rounds) {
  const int n = d * d;
  const size_t elem = dtype == SV_C128 ? 16 : 8;
  const size_t ns = (size_t)d * d - 1;
  const size_t per_traj = sizeof(BlockRT) * (size_t)rounds * ns;
  const size_t table = std::min<size_t>((size_t)n_traj * per_traj, std::max<size_t>(per_traj, (size_t)64 << 20));
  // two registers: a speculative run writes the other buffer each pass
  return (2 * elem << n) + table + (size_t)n_traj * (rounds * ns + n) + (sizeof(double) << (n > 12 ? n - 12 : 0)) +
         (2u << 20);
}

sv_status check_job(const sv_job* job) {
  if (!job) return fail(SV_EINVAL, "NULL job");
  if (job->d < 2 || job->d > 5) return fail(SV_EINVAL, "d=%d out of 2..5", job->d);
  if (job->gateset != SV_GATESET_CR && job->gateset != SV_GATESET_TEXTBOOK)
    return fail(SV_EINVAL, "bad gateset %d", job->gateset);
  if (job->rounds < 1 || job->rounds > 100000) return fail(SV_EINVAL, "rounds=%d", job->rounds);
  if (job->dtype != SV_C64 && job->dtype != SV_C128) return fail(SV_EINVAL, "bad dtype");
  if (job->n_traj < 1) return fail(SV_EINVAL, "n_traj must be >= 1");
  if (job->flags != 0) return fail(SV_EINVAL, "flags must be 0");
  if (!(job->p >= 0.0 && job->p <= 1.0)) return fail(SV_EINVAL, "p out of [0, 1]");
  if (!std::isfinite(job->eps) || !std::isfinite(job->zeta)) return fail(SV_EINVAL, "non-finite eps/zeta");
  return SV_OK;
}

struct SJob {
  uint64_t tag = 0;
  sv_job job{};
  std::vector<double> eps;  // one exponent per gate site
  uint8_t* records = nullptr;
  uint8_t* bits = nullptr;
  double t_submit = 0, t_admit = 0;
  size_t cost = 0;
  int status = SV_OK;
  int dispatched = 0;
  int finished = 0;
  int n_stab = 0;
};

struct LaneKey {
  int d, gateset, dtype;
  double zeta;
  bool operator<(const LaneKey& o) const {
    if (d != o.d) return d < o.d;
    if (gateset != o.gateset) return gateset < o.gateset;
    if (dtype != o.dtype) return dtype < o.dtype;
    return zeta < o.zeta;
  }
};

struct Piece {
  SJob* job;
  int first, count;
};

}  // namespace

struct sv_server_s {
  sv_server_config cfg{};
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  std::condition_variable cv_idle;
  std::deque<SJob*> pending;
  std::deque<SJob*> big;
  std::map<LaneKey, std::deque<SJob*>> lanes;
  std::vector<sv_completion> done;
  size_t used = 0, high = 0;
  int running = 0, completed = 0, launches = 0, in_system = 0;
  std::atomic<int> cancel{0};
  bool stop = false;
  std::vector<std::thread> threads;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  void finish_locked(SJob* j, int status) {
    used -= j->cost;
    ++completed;
    --in_system;
    sv_completion c{};
    c.tag = j->tag;
    c.status = status;
    c.t_submit = j->t_submit;
    c.t_admit = j->t_admit;
    c.t_done = now();
    done.push_back(c);
    delete j;
    cv_idle.notify_all();
  }

  void admit_locked() {
    while (!pending.empty()) {
      SJob* j = pending.front();
      if (used > 0 && used + j->cost > cfg.hbm_budget) break;
      pending.pop_front();
      used += j->cost;
      high = std::max(high, used);
      j->t_admit = now();
      if (j->job.d >= 5) {
        big.push_back(j);
      } else {
        const LaneKey k{j->job.d, j->job.gateset, j->job.dtype, j->job.zeta};
        auto it = lanes.find(k);
        if (it == lanes.end()) {
          lanes[k];
          threads.emplace_back([this, k] { lane_worker(k); });
        }
        lanes[k].push_back(j);
      }
    }
    cv.notify_all();
  }

  void big_worker() {
    (void)hipSetDevice(device);
    hipStream_t hs = nullptr;
    (void)hipStreamCreateWithFlags(&hs, hipStreamNonBlocking);
    for (;;) {
      SJob* j = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !big.empty(); });
        if (big.empty()) break;
        j = big.front();
        big.pop_front();
        ++running;
      }
      sv_job job = j->job;
      job.hip_stream = hs;
      job.eps_site = j->eps.data();
      sv_result res{};
      res.records = j->records;
      res.final_bits = j->bits;
      sv_status st;
      if (cancel.load()) {
        st = SV_EBUSY;
      } else {
        const Template tp = build_template(job.d, job.gateset);
        st = job.dtype == SV_C128 ? run_rounds_t<double>(&job, &res, tp, &cancel)
                                  : run_rounds_t<float>(&job, &res, tp, &cancel);
      }
      std::lock_guard<std::mutex> lk(mu);
      --running;
      ++launches;
      finish_locked(j, st);
      admit_locked();
    }
    (void)hipStreamDestroy(hs);
  }

  void lane_worker(LaneKey key) {
    (void)hipSetDevice(device);
    hipStream_t hs = nullptr;
    (void)hipStreamCreateWithFlags(&hs, hipStreamNonBlocking);
    const Template tp = build_template(key.d, key.gateset);
    const int n = key.d * key.d, ns = (int)tp.blocks.size();
    for (;;) {
      std::vector<Piece> pieces;
      int total = 0, max_rounds = 1;
      {
        std::unique_lock<std::mutex> lk(mu);
        auto& q = lanes[key];
        cv.wait(lk, [&] { return stop || !q.empty(); });
        if (q.empty()) break;
        while (!q.empty() && total < cfg.max_batch_traj) {
          SJob* j = q.front();
          const int take = std::min(j->job.n_traj - j->dispatched, cfg.max_batch_traj - total);
          pieces.push_back({j, j->dispatched, take});
          j->dispatched += take;
          total += take;
          max_rounds = std::max(max_rounds, j->job.rounds);
          if (j->dispatched == j->job.n_traj) q.pop_front();
        }
        ++running;
      }
      std::vector<uint64_t> seeds(total), streams(total);
      std::vector<int> rounds(total);
      std::vector<double> p(total), eps((size_t)total * tp.n_sites);
      int at = 0;
      for (const Piece& pc : pieces)
        for (int i = 0; i < pc.count; ++i, ++at) {
          seeds[at] = pc.job->job.seed;
          streams[at] = pc.job->job.traj0 + (uint64_t)(pc.first + i);
          rounds[at] = pc.job->job.rounds;
          p[at] = pc.job->job.p;
          std::copy(pc.job->eps.begin(), pc.job->eps.end(), eps.begin() + (size_t)at * tp.n_sites);
        }
      std::vector<uint8_t> rec((size_t)total * max_rounds * ns), bits((size_t)total * n);
      BatchInputs in{key.d, key.gateset, total, max_rounds, key.zeta, seeds.data(), streams.data(),
                     rounds.data(), p.data(), eps.data(), tp.n_sites, rec.data(), bits.data(), hs, 0.0};
      sv_status st = SV_EBUSY;
      if (!cancel.load())
        st = key.dtype == SV_C128 ? run_batch_core<double>(in, tp) : run_batch_core<float>(in, tp);
      std::lock_guard<std::mutex> lk(mu);
      --running;
      ++launches;
      at = 0;
      for (const Piece& pc : pieces) {
        SJob* j = pc.job;
        for (int i = 0; i < pc.count; ++i, ++at) {
          const int t = pc.first + i;
          if (st == SV_OK) {
            std::memcpy(j->records + (size_t)t * j->job.rounds * ns, rec.data() + (size_t)at * max_rounds * ns,
                        (size_t)j->job.rounds * ns);
            std::memcpy(j->bits + (size_t)t * n, bits.data() + (size_t)at * n, n);
          }
        }
        if (st != SV_OK) j->status = st;
        j->finished += pc.count;
        if (j->finished == j->job.n_traj) finish_locked(j, j->status);
      }
      admit_locked();
    }
    (void)hipStreamDestroy(hs);
  }
};

extern "C" {

sv_status sv_server_create(const sv_server_config* cfg, sv_server* out) {
  if (!cfg || !out) return fail(SV_EINVAL, "NULL argument");
  if (cfg->big_streams < 1 || cfg->big_streams > 16) return fail(SV_EINVAL, "big_streams out of 1..16");
  if (cfg->max_batch_traj < 1) return fail(SV_EINVAL, "max_batch_traj must be >= 1");
  if (cfg->hbm_budget == 0) return fail(SV_EINVAL, "hbm_budget must be > 0");
  if (cfg->flags != 0) return fail(SV_EINVAL, "flags must be 0");
  sv_server s = new (std::nothrow) sv_server_s;
  if (!s) return fail(SV_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  s->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(SV_EDEVICE, "no HIP device");
  }
  for (int i = 0; i < cfg->big_streams; ++i) s->threads.emplace_back([s] { s->big_worker(); });
  *out = s;
  return SV_OK;
}

sv_status sv_server_submit(sv_server s, const sv_request* req) {
  if (!s || !req) return fail(SV_EINVAL, "NULL argument");
  sv_status st = check_job(&req->job);
  if (st != SV_OK) return st;
  if (!req->records || !req->final_bits) return fail(SV_EINVAL, "records and final_bits are required");
  const Template tp = build_template(req->job.d, req->job.gateset);
  SJob* j = new (std::nothrow) SJob;
  if (!j) return fail(SV_ENOMEM, "host allocation failed");
  j->tag = req->tag;
  j->job = req->job;
  j->job.hip_stream = nullptr;
  j->records = req->records;
  j->bits = req->final_bits;
  j->n_stab = (int)tp.blocks.size();
  j->eps.assign(std::max(1, tp.n_sites), req->job.eps);
  if (req->job.eps_site)
    for (int i = 0; i < tp.n_sites; ++i) {
      if (!std::isfinite(req->job.eps_site[i])) {
        delete j;
        return fail(SV_EINVAL, "non-finite eps_site[%d]", i);
      }
      j->eps[i] = req->job.eps_site[i];
    }
  j->job.eps_site = nullptr;
  j->cost = req->job.d >= 5
                ? rounds_footprint(req->job.d, req->job.dtype, req->job.n_traj, req->job.rounds)
                : batch_footprint(req->job.d, req->job.dtype, req->job.n_traj, req->job.rounds, tp.n_sites);
  if (j->cost > s->cfg.hbm_budget) {
    const size_t c = j->cost;
    delete j;
    return fail(SV_ENOMEM, "job needs %zu device bytes > budget %zu", c, s->cfg.hbm_budget);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    delete j;
    return fail(SV_EBUSY, "server is shutting down");
  }
  j->t_submit = s->now();
  ++s->in_system;
  s->pending.push_back(j);
  s->admit_locked();
  return SV_OK;
}

int sv_server_poll(sv_server s, sv_completion* out, int max) {
  if (!s || !out || max <= 0) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  const int k = std::min<int>(max, (int)s->done.size());
  for (int i = 0; i < k; ++i) out[i] = s->done[i];
  s->done.erase(s->done.begin(), s->done.begin() + k);
  return k;
}

sv_status sv_server_wait_idle(sv_server s, double timeout_s) {
  if (!s) return fail(SV_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  const bool ok = s->cv_idle.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                      [&] { return s->in_system == 0; });
  return ok ? SV_OK : fail(SV_EBUSY, "server still busy after %.1f s", timeout_s);
}

sv_status sv_server_stats_get(sv_server s, sv_server_stats* out) {
  if (!s || !out) return fail(SV_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out->hbm_in_use = s->used;
  out->hbm_high_water = s->high;
  out->pending = (int)s->pending.size();
  out->running = s->running;
  out->completed = s->completed;
  out->launches = s->launches;
  return SV_OK;
}

double sv_server_clock(sv_server s) { return s ? s->now() : 0.0; }

sv_status sv_server_destroy(sv_server s, int cancel) {
  if (!s) return SV_OK;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    if (cancel) {
      // queued jobs end now; admitted ones end at their next trajectory or launch
      s->cancel.store(1);
      while (!s->pending.empty()) {
        SJob* j = s->pending.front();
        s->pending.pop_front();
        s->used += j->cost;  // finish_locked releases it
        s->finish_locked(j, SV_EBUSY);
      }
    }
    s->cv_idle.wait(lk, [&] { return s->in_system == 0; });
    s->stop = true;
  }
  s->cv.notify_all();
  std::vector<std::thread> ts;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    ts.swap(s->threads);
  }
  for (auto& t : ts) t.join();
  delete s;
  return SV_OK;
}

}  // extern "C"

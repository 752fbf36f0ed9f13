// Request serving: compress (Alg. 1 with adaptive sampling) + ULV factor
// (Alg. 3) + solve (Alg. 4) for requests that arrive over time, and
// solve-only requests against handles kept resident on the device.
//
// Requests wait in arrival order.  Each worker thread owns a HIP stream; a
// free worker admits the oldest waiting request it can run and, behind it,
// the waiting requests of the same kind: compress requests with the same
// storage type and options (compressed together by one batched compression,
// then factored and solved one by one), or solve-only requests on distinct
// resident handles (queued back to back on the worker's stream), while their
// device footprint fits the budget.  Resident handles count with their
// device bytes until they are released.  Requests that arrive meanwhile are
// admitted by the next free worker as memory frees up, so their work
// overlaps on the device with the batches already running.  A request whose
// footprint alone exceeds the budget runs when nothing else is admitted.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hss_handle.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  long long id = 0;
  const void* A = nullptr;  // null: solve-only request on `on`
  int dtype = HSS_F64;
  long long n = 0, lda = 0;
  hss_opts opts{};
  hss_handle on = nullptr;  // solve-only: the resident handle
  bool keep = false;        // compress: keep the handle resident
  int nrhs = 0;
  const double* b = nullptr;
  long long ldb = 0;
  double* x = nullptr;
  long long ldx = 0;
  long long footprint = 0;
  hipEvent_t ready = nullptr;  // recorded on the submitter's stream: A and b are written
  hss_request_info info{};
  bool done = false;
};

bool same_opts(const Req& a, const Req& b) {
  const hss_opts &p = a.opts, &q = b.opts;
  return a.dtype == b.dtype && p.rtol == q.rtol && p.d0 == q.d0 && p.dd == q.dd &&
         p.d_max == q.d_max && p.p_margin == q.p_margin && p.seed == q.seed &&
         p.leaf_size == q.leaf_size && p.sample_prec == q.sample_prec;
}

// Device bytes a compress request holds while it runs: its inputs and
// outputs (A, b, x), the compression's random matrices, samples and local
// samples (about 8 n d_max doubles), the generators and ULV factors with the
// solve's compact-WY reflector blocks (a few n x leaf blocks), the solve
// workspace and slack.
long long compress_footprint(long long n, long long lda, int dtype, int nrhs, const hss_opts& o) {
  const long long ldg = (o.d_max + 7) / 8 * 8;
  const long long a_bytes = n * lda * (dtype == HSS_F32 ? 4 : 8);
  const long long rhs_bytes = 2LL * n * nrhs * 8;
  return a_bytes + rhs_bytes + 8LL * n * ldg * 8 + 8LL * n * std::max(o.leaf_size, 1) * 8 +
         4LL * n * nrhs * 8 + (64LL << 20);
}

// A solve-only request: b, x and the solve workspace (four vectors of the
// node dimension per node, about 4 n nrhs doubles over a level, a few levels
// at once) and slack.
long long solve_footprint(long long n, int nrhs) { return 2LL * n * nrhs * 8 + 16LL * n * nrhs * 8 + (4LL << 20); }

struct Resident {
  long long bytes = 0;
  bool busy = false;       // a request on it is running
  bool releasing = false;  // hss_server_release is waiting for it
};

}  // namespace

struct hss_server_s {
  hss_server_opts o{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<long long> queue;
  std::unordered_map<long long, std::unique_ptr<Req>> reqs;
  std::unordered_map<hss_handle, Resident> resident;
  long long next_id = 1;
  long long in_use = 0;  // admitted requests plus resident handles
  int running = 0;       // admitted requests
  bool stop = false;
  std::vector<std::thread> workers;
  Clock::time_point t0 = Clock::now();

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  // requests waiting or running on resident handle h (lock held)
  bool has_requests_on(hss_handle h) {
    for (long long id : queue)
      if (reqs[id]->on == h) return true;
    auto it = resident.find(h);
    return it != resident.end() && it->second.busy;
  }

  // The requests a free worker takes now (lock held); empty if none can
  // run.  The oldest request that can run (a solve-only request waits while
  // its handle is busy) decides the kind of the batch; it is admitted if it
  // fits the budget or nothing else runs, and the later ones of its kind
  // join while they fit.  Nothing changes when the result is empty.
  std::vector<Req*> admit() {
    std::vector<Req*> batch;
    long long used = in_use;
    Req* head = nullptr;
    for (long long id : queue) {
      Req* r = reqs[id].get();
      bool take = false;
      if (r->on) {
        auto it = resident.find(r->on);
        const bool free_handle = it != resident.end() && !it->second.busy;
        bool dup = false;  // one request per handle in a batch
        for (Req* q : batch) dup = dup || q->on == r->on;
        if (free_handle && !dup) {
          if (!head) take = running == 0 || used + r->footprint <= o.hbm_budget;
          else take = head->on && used + r->footprint <= o.hbm_budget && (int)batch.size() < o.max_batch;
        }
      } else {
        if (!head) take = running == 0 || used + r->footprint <= o.hbm_budget;
        else take = !head->on && used + r->footprint <= o.hbm_budget && (int)batch.size() < o.max_batch &&
                    same_opts(*r, *head);
      }
      if (!head && !take && !r->on) break;  // the oldest compress request waits for memory: keep order
      if (take) {
        if (!head) head = r;
        batch.push_back(r);
        used += r->footprint;
        if (r->on) resident[r->on].busy = true;
      }
    }
    if (batch.empty()) return batch;
    // requests behind the stopping point stay queued in order
    std::deque<long long> rest;
    for (long long id : queue) {
      bool taken = false;
      for (Req* r : batch) taken = taken || r->id == id;
      if (!taken) rest.push_back(id);
    }
    queue.swap(rest);
    in_use = used;
    running += (int)batch.size();
    return batch;
  }

  void finish(const std::vector<Req*>& batch, const std::vector<long long>& kept_bytes) {
    std::lock_guard<std::mutex> lk(mu);
    const double t = now();
    for (size_t i = 0; i < batch.size(); ++i) {
      Req* r = batch[i];
      in_use -= r->footprint;
      if (r->on) {
        Resident& rs = resident[r->on];
        rs.busy = false;
        const long long b = hss::resident_bytes(r->on->h);  // the solve workspace may have grown
        in_use += b - rs.bytes;
        rs.bytes = b;
      }
      if (r->info.handle) {  // kept resident: counts with its actual bytes
        resident[r->info.handle] = Resident{kept_bytes[i], false, false};
        in_use += kept_bytes[i];
      }
      r->info.t_done = t;
      r->done = true;
    }
    running -= (int)batch.size();
    cv_done.notify_all();
    cv_work.notify_all();
  }

  void run_compress(const std::vector<Req*>& batch, hipStream_t s, std::vector<long long>& kept_bytes) {
    const int nb = (int)batch.size();
    std::vector<const void*> As(nb);
    std::vector<long long> ns(nb), ldas(nb);
    bool any_keep = false;
    for (int i = 0; i < nb; ++i) {
      As[i] = batch[i]->A;
      ns[i] = batch[i]->n;
      ldas[i] = batch[i]->lda;
      any_keep = any_keep || batch[i]->keep;
    }
    std::vector<hss_handle> hs(nb, nullptr);
    std::vector<int> st(nb, HSS_OK);
    // a kept handle outlives the others of its batch: separate generator arenas
    const hss_status cs = hss::compress_batched(nb, As.data(), batch[0]->dtype, ns.data(), ldas.data(), nullptr,
                                                &batch[0]->opts, s, hs.data(), st.data(), !any_keep);
    if (cs != HSS_OK && cs != HSS_NOT_CONVERGED) {
      for (Req* r : batch) r->info.status = cs;
      return;
    }
    for (int i = 0; i < nb; ++i) {
      Req* r = batch[i];
      hss_status f = hss_factor(hs[i], s);
      if (f == HSS_OK && r->nrhs > 0) f = hss_solve(hs[i], r->nrhs, r->b, r->ldb, r->x, r->ldx, s);
      r->info.status = f != HSS_OK ? f : st[i];
      hss_stats_t stt{};
      if (hss_stats(hs[i], &stt) == HSS_OK) {
        r->info.d_final = stt.d_final;
        r->info.max_rank = stt.max_rank;
      }
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
      (void)hipGetLastError();
      for (Req* r : batch)
        if (r->info.status == HSS_OK || r->info.status == HSS_NOT_CONVERGED) r->info.status = HSS_ERR_HIP;
    }
    for (int i = 0; i < nb; ++i) {
      Req* r = batch[i];
      const bool ok = r->info.status == HSS_OK || r->info.status == HSS_NOT_CONVERGED;
      if (r->keep && ok) {
        r->info.handle = hs[i];
        kept_bytes[i] = hss::resident_bytes(hs[i]->h);
      } else {
        hss_destroy(hs[i]);
      }
    }
  }

  void run_solve(const std::vector<Req*>& batch, hipStream_t s) {
    for (Req* r : batch) {  // stream-ordered: queued back to back, one wait
      r->info.status = hss_solve(r->on, r->nrhs, r->b, r->ldb, r->x, r->ldx, s);
      hss_stats_t stt{};
      if (hss_stats(r->on, &stt) == HSS_OK) {
        r->info.d_final = stt.d_final;
        r->info.max_rank = stt.max_rank;
      }
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
      (void)hipGetLastError();
      for (Req* r : batch)
        if (r->info.status == HSS_OK) r->info.status = HSS_ERR_HIP;
    }
  }

  void run(const std::vector<Req*>& batch, hipStream_t s, std::vector<long long>& kept_bytes) {
    for (Req* r : batch) {  // the inputs are read only after the submitter wrote them
      r->info.batch_size = (int)batch.size();
      if (r->ready) {
        hss::order_after(s, r->ready);
        (void)hipEventDestroy(r->ready);
        r->ready = nullptr;
      }
    }
    if (batch[0]->on) run_solve(batch, s);
    else run_compress(batch, s, kept_bytes);
  }

  void worker() {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    while (true) {
      std::vector<Req*> batch;
      {
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
          if (stop && queue.empty()) break;
          batch = admit();
          if (!batch.empty()) break;
          cv_work.wait(lk);
        }
        if (batch.empty()) break;
        const double t = now();
        for (Req* r : batch) r->info.t_start = t;
      }
      std::vector<long long> kept(batch.size(), 0);
      if (!s) {
        for (Req* r : batch) r->info.status = HSS_ERR_HIP;
      } else {
        run(batch, s, kept);
      }
      finish(batch, kept);
    }
    if (s) (void)hipStreamDestroy(s);
  }
};

extern "C" {

void hss_server_default_opts(hss_server_opts* o) {
  if (!o) return;
  o->hbm_budget = 0;
  o->max_batch = 32;
  o->workers = 2;
}

hss_status hss_server_create(const hss_server_opts* opts, hss_server* out) {
  if (!out) return hss::set_error(HSS_ERR_ARG, "out is NULL");
  *out = nullptr;
  hss_server_opts o;
  if (opts) o = *opts;
  else hss_server_default_opts(&o);
  if (o.max_batch < 1 || o.workers < 1 || o.workers > 16 || o.hbm_budget < 0)
    return hss::set_error(HSS_ERR_ARG, "max_batch / workers / hbm_budget");
  if (o.hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return hss::set_error(HSS_ERR_HIP, "hipMemGetInfo");
    o.hbm_budget = (long long)(0.8 * (double)tot);
  }
  hss_server_s* sv = new (std::nothrow) hss_server_s();
  if (!sv) return hss::set_error(HSS_ERR_ALLOC, "server");
  sv->o = o;
  for (int w = 0; w < o.workers; ++w) sv->workers.emplace_back([sv] { sv->worker(); });
  *out = sv;
  return HSS_OK;
}

hss_status hss_server_submit_request(hss_server sv, const hss_server_request* q, void* stream,
                                     long long* ticket) {
  if (!sv || !q || !ticket) return hss::set_error(HSS_ERR_ARG, "server, request or ticket is NULL");
  auto r = std::make_unique<Req>();
  if (q->handle) {
    if (q->A) return hss::set_error(HSS_ERR_ARG, "a request has either A or a resident handle");
    if (q->nrhs < 1 || !q->b || !q->x || q->ldb < q->nrhs || q->ldx < q->nrhs)
      return hss::set_error(HSS_ERR_ARG, "nrhs, b, x, ldb or ldx invalid");
    r->on = q->handle;
    r->n = q->handle->h.n;
  } else {
    if (!q->A || q->n < 1 || q->lda < q->n || (q->dtype != HSS_F64 && q->dtype != HSS_F32))
      return hss::set_error(HSS_ERR_ARG, "A, n, lda or dtype invalid");
    if (q->nrhs < 0 || (q->nrhs > 0 && (!q->b || !q->x || q->ldb < q->nrhs || q->ldx < q->nrhs)))
      return hss::set_error(HSS_ERR_ARG, "nrhs, b, x, ldb or ldx invalid");
    r->A = q->A;
    r->dtype = q->dtype;
    r->n = q->n;
    r->lda = q->lda;
    if (q->opts) r->opts = *q->opts;
    else hss_default_opts(&r->opts);
    if (r->opts.R_user_r || r->opts.R_user_c)
      return hss::set_error(HSS_ERR_ARG, "no user random matrices in served requests");
    if (r->opts.sample_prec != HSS_SAMPLE_F64 && q->dtype != HSS_F32)
      return hss::set_error(HSS_ERR_ARG, "reduced-precision sampling needs A stored in FP32");
    r->keep = q->keep != 0;
  }
  r->nrhs = q->nrhs;
  r->b = q->b;
  r->ldb = q->ldb;
  r->x = q->x;
  r->ldx = q->ldx;
  r->footprint = r->on ? solve_footprint(r->n, r->nrhs)
                       : compress_footprint(r->n, r->lda, r->dtype, r->nrhs, r->opts);
  if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(r->ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
    if (r->ready) (void)hipEventDestroy(r->ready);
    return hss::set_error(HSS_ERR_HIP, "event on the submitting stream");
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    hss_status bad = HSS_OK;
    if (sv->stop) bad = hss::set_error(HSS_ERR_STATE, "server is shutting down");
    if (r->on) {
      auto it = sv->resident.find(r->on);
      if (it == sv->resident.end() || it->second.releasing)
        bad = hss::set_error(HSS_ERR_ARG, "the handle is not resident in this server");
    }
    if (bad != HSS_OK) {
      (void)hipEventDestroy(r->ready);
      return bad;
    }
    r->id = sv->next_id++;
    r->info.t_submit = sv->now();
    r->info.status = HSS_OK;
    *ticket = r->id;
    sv->queue.push_back(r->id);
    sv->reqs[r->id] = std::move(r);
  }
  sv->cv_work.notify_all();
  return HSS_OK;
}

hss_status hss_server_submit(hss_server sv, const void* A, int dtype, long long n, long long lda,
                             const hss_opts* opts, int nrhs, const double* b, long long ldb,
                             double* x, long long ldx, void* stream, long long* ticket) {
  hss_server_request q{};
  q.A = A;
  q.dtype = dtype;
  q.n = n;
  q.lda = lda;
  q.opts = opts;
  q.nrhs = nrhs;
  q.b = b;
  q.ldb = ldb;
  q.x = x;
  q.ldx = ldx;
  if (!A) return hss::set_error(HSS_ERR_ARG, "A, n, lda or dtype invalid");
  return hss_server_submit_request(sv, &q, stream, ticket);
}

hss_status hss_server_wait(hss_server sv, long long ticket, hss_request_info* info) {
  if (!sv) return hss::set_error(HSS_ERR_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return hss::set_error(HSS_ERR_ARG, "unknown ticket");
  Req* r = it->second.get();
  sv->cv_done.wait(lk, [&] { return r->done; });
  if (info) *info = r->info;
  const hss_status st = (hss_status)r->info.status;
  sv->reqs.erase(it);
  if (st != HSS_OK && st != HSS_NOT_CONVERGED) return hss::set_error(st, "request failed");
  return st;
}

hss_status hss_server_release(hss_server sv, hss_handle h) {
  if (!sv || !h) return hss::set_error(HSS_ERR_ARG, "server or handle is NULL");
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->resident.find(h);
    if (it == sv->resident.end() || it->second.releasing)
      return hss::set_error(HSS_ERR_ARG, "the handle is not resident in this server");
    it->second.releasing = true;
    sv->cv_done.wait(lk, [&] { return !sv->has_requests_on(h); });
    sv->in_use -= sv->resident[h].bytes;
    sv->resident.erase(h);
  }
  hss_destroy(h);
  sv->cv_work.notify_all();
  return HSS_OK;
}

void hss_server_destroy(hss_server sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (std::thread& t : sv->workers) t.join();
  for (auto& kv : sv->resident) hss_destroy(kv.first);
  delete sv;
}

}  // extern "C"

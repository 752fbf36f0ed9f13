// Request serving: compress (Alg. 1 with adaptive sampling) + ULV factor
// (Alg. 3) + solve (Alg. 4) for requests that arrive over time.
//
// Requests wait in arrival order.  Each worker thread owns a HIP stream; a
// free worker admits the oldest waiting request and, behind it, the waiting
// requests compatible with it (same storage type and compression options)
// while their estimated device footprint fits the budget, compresses them
// together with one batched compression, then factors and solves each, and
// frees their footprint.  Requests that arrive meanwhile are admitted by the
// next free worker as memory frees up, so their work overlaps on the device
// with the batches already running.  A request whose footprint alone exceeds
// the budget runs when nothing else is admitted.
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
  const void* A = nullptr;
  int dtype = HSS_F64;
  long long n = 0, lda = 0;
  hss_opts opts{};
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

// Device bytes a request holds while it runs: the compression's random
// matrices, samples and local samples (about 8 n d_max doubles), the
// generators and ULV factors (a few n x leaf blocks) and slack.
long long footprint_of(long long n, const hss_opts& o) {
  const long long ldg = (o.d_max + 7) / 8 * 8;
  return 8LL * n * ldg * 8 + 6LL * n * std::max(o.leaf_size, 1) * 8 + (64LL << 20);
}

}  // namespace

struct hss_server_s {
  hss_server_opts o{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<long long> queue;
  std::unordered_map<long long, std::unique_ptr<Req>> reqs;
  long long next_id = 1;
  long long in_use = 0;
  int running = 0;  // admitted requests
  bool stop = false;
  std::vector<std::thread> workers;
  Clock::time_point t0 = Clock::now();

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  // the requests a free worker takes now (lock held); empty if none fits
  std::vector<Req*> admit() {
    std::vector<Req*> batch;
    if (queue.empty()) return batch;
    Req* head = reqs[queue.front()].get();
    if (running > 0 && in_use + head->footprint > o.hbm_budget) return batch;
    long long used = in_use;
    std::deque<long long> keep;
    for (long long id : queue) {
      Req* r = reqs[id].get();
      const bool fits = batch.empty() || (used + r->footprint <= o.hbm_budget &&
                                          (int)batch.size() < o.max_batch && same_opts(*r, *head));
      if (fits) {
        batch.push_back(r);
        used += r->footprint;
      } else {
        keep.push_back(id);
      }
    }
    queue.swap(keep);
    in_use = used;
    running += (int)batch.size();
    return batch;
  }

  void finish(const std::vector<Req*>& batch) {
    std::lock_guard<std::mutex> lk(mu);
    const double t = now();
    for (Req* r : batch) {
      in_use -= r->footprint;
      r->info.t_done = t;
      r->done = true;
    }
    running -= (int)batch.size();
    cv_done.notify_all();
    cv_work.notify_all();
  }

  void run(const std::vector<Req*>& batch, hipStream_t s) {
    const int nb = (int)batch.size();
    for (Req* r : batch)  // the inputs are read only after the submitter wrote them
      if (r->ready) {
        hss::order_after(s, r->ready);
        (void)hipEventDestroy(r->ready);
        r->ready = nullptr;
      }
    std::vector<const void*> As(nb);
    std::vector<long long> ns(nb), ldas(nb);
    for (int i = 0; i < nb; ++i) {
      As[i] = batch[i]->A;
      ns[i] = batch[i]->n;
      ldas[i] = batch[i]->lda;
      batch[i]->info.batch_size = nb;
    }
    std::vector<hss_handle> hs(nb, nullptr);
    std::vector<int> st(nb, HSS_OK);
    const hss_status cs = hss_compress_batched(nb, As.data(), batch[0]->dtype, ns.data(), ldas.data(),
                                               nullptr, &batch[0]->opts, s, hs.data(), st.data());
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
    (void)hipStreamSynchronize(s);
    for (hss_handle h : hs) hss_destroy(h);
  }

  void worker() {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    while (true) {
      std::vector<Req*> batch;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          if (stop && queue.empty()) return true;
          if (queue.empty()) return false;
          const Req* head = reqs[queue.front()].get();
          return running == 0 || in_use + head->footprint <= o.hbm_budget;
        });
        if (stop && queue.empty()) break;
        batch = admit();
        const double t = now();
        for (Req* r : batch) r->info.t_start = t;
      }
      if (batch.empty()) continue;
      if (!s) {
        for (Req* r : batch) r->info.status = HSS_ERR_HIP;
      } else {
        run(batch, s);
      }
      finish(batch);
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

hss_status hss_server_submit(hss_server sv, const void* A, int dtype, long long n, long long lda,
                             const hss_opts* opts, int nrhs, const double* b, long long ldb,
                             double* x, long long ldx, void* stream, long long* ticket) {
  if (!sv || !ticket) return hss::set_error(HSS_ERR_ARG, "server or ticket is NULL");
  if (!A || n < 1 || lda < n || (dtype != HSS_F64 && dtype != HSS_F32))
    return hss::set_error(HSS_ERR_ARG, "A, n, lda or dtype invalid");
  if (nrhs < 0 || (nrhs > 0 && (!b || !x || ldb < nrhs || ldx < nrhs)))
    return hss::set_error(HSS_ERR_ARG, "nrhs, b, x, ldb or ldx invalid");
  auto r = std::make_unique<Req>();
  r->A = A;
  r->dtype = dtype;
  r->n = n;
  r->lda = lda;
  if (opts) r->opts = *opts;
  else hss_default_opts(&r->opts);
  if (r->opts.R_user_r || r->opts.R_user_c)
    return hss::set_error(HSS_ERR_ARG, "no user random matrices in served requests");
  if (r->opts.sample_prec != HSS_SAMPLE_F64 && dtype != HSS_F32)
    return hss::set_error(HSS_ERR_ARG, "reduced-precision sampling needs A stored in FP32");
  r->nrhs = nrhs;
  r->b = b;
  r->ldb = ldb;
  r->x = x;
  r->ldx = ldx;
  r->footprint = footprint_of(n, r->opts);
  if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(r->ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
    if (r->ready) (void)hipEventDestroy(r->ready);
    return hss::set_error(HSS_ERR_HIP, "event on the submitting stream");
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      (void)hipEventDestroy(r->ready);
      return hss::set_error(HSS_ERR_STATE, "server is shutting down");
    }
    r->id = sv->next_id++;
    r->info.t_submit = sv->now();
    r->info.status = HSS_OK;
    *ticket = r->id;
    sv->queue.push_back(r->id);
    sv->reqs[r->id] = std::move(r);
  }
  sv->cv_work.notify_one();
  return HSS_OK;
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

void hss_server_destroy(hss_server sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (std::thread& t : sv->workers) t.join();
  delete sv;
}

}  // extern "C"

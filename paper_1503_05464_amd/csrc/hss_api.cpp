// C ABI of the randomized HSS library: compression (Alg. 1 with the
// late-notification adaptive sampling of Alg. 5, run level-synchronously over
// node heights), HSS matvec (Alg. 2), export / import of generators and the
// exported building blocks.  The ULV factorization and solve are in
// hss_ulv.cpp.  All arithmetic runs in the HIP kernels; this file sizes
// buffers, builds descriptor tables and orders the launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "hss_handle.h"

using namespace hss;

namespace {

thread_local std::string g_err;

hss_status fail(hss_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

}  // namespace

hss_status hss::set_error(hss_status st, const std::string& msg) { return fail(st, msg); }

namespace {

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      return fail(HSS_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define CHK(x)                              \
  do {                                      \
    hss_status st_ = (x);                   \
    if (st_ != HSS_OK) return st_;          \
  } while (0)

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int verbose_level(const char* v) {
  if (!v || !v[0] || v[0] == '0') return 0;
  return (v[0] >= '1' && v[0] <= '9') ? v[0] - '0' : 1;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

// ---------------------------------------------------------------------------
// memory helpers
// ---------------------------------------------------------------------------
namespace hss {

namespace {
// Freed device blocks of 1 MB and more are kept for reuse, by size class (four
// classes per power of two), up to a quarter of the device's memory: the
// runtime pool returns freed memory to the system at synchronizations, and
// mapping it again can take seconds when a step frees and allocates tens of
// GB (batched compressions).  A reused block is ordered after its last use
// by an event recorded when it was freed.  Blocks are kept per device.
struct CachedBlock {
  void* p;
  hipEvent_t ev;  // recorded on the freeing stream
};
struct LiveBlock {
  size_t cls;
  int dev;
};
std::mutex g_dev_mu;
std::unordered_map<unsigned long long, std::vector<CachedBlock>> g_dev_free;  // by (class, device)
std::unordered_map<void*, LiveBlock> g_dev_live;  // cached-size blocks in use
size_t g_dev_cached = 0;
size_t g_dev_cap = 0;
std::once_flag g_dev_once;

}  // namespace

// Orders stream s after event ev: a device-side wait, or, when that cannot be
// queued, a host-side wait for ev (the same ordering, coarser).
void order_after(hipStream_t s, hipEvent_t ev) {
  if (hipStreamWaitEvent(s, ev, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventSynchronize(ev);
  }
}

namespace {
unsigned long long cache_key(size_t cls, int dev) { return ((unsigned long long)cls << 8) | (unsigned)(dev & 255); }

constexpr size_t kCacheMin = (size_t)1 << 20;

size_t size_class(size_t b) {
  if (b < kCacheMin) return 0;
  size_t top = kCacheMin;
  while (top * 2 <= b) top *= 2;
  const size_t step = top / 4;
  return (b + step - 1) / step * step;
}

// frees every cached block of device dev, each after its last use, on
// stream s of that device (lock held)
void trim_cache(int dev, hipStream_t s) {
  for (auto it = g_dev_free.begin(); it != g_dev_free.end();) {
    if ((int)(it->first & 255) != (dev & 255)) {
      ++it;
      continue;
    }
    const size_t cls = (size_t)(it->first >> 8);
    for (CachedBlock& c : it->second) {
      order_after(s, c.ev);
      (void)hipEventDestroy(c.ev);
      (void)hipFreeAsync(c.p, s);
      g_dev_cached -= cls;
    }
    it = g_dev_free.erase(it);
  }
}
}  // namespace

namespace {
// A caller-supplied allocator (hss_set_allocator).  Blocks remember the
// allocator that made them, so changing allocators while blocks are live is
// safe: each goes back where it came from.
struct UserAlloc {
  hss_alloc_fn alloc = nullptr;
  hss_free_fn free = nullptr;
  void* ctx = nullptr;
};
struct UserBlock {
  size_t bytes;
  int dev;
  hipStream_t stream;  // the stream the block was allocated for
  UserAlloc ua;
};
std::mutex g_user_mu;
UserAlloc g_user;
std::unordered_map<void*, UserBlock> g_user_live;

void* user_alloc(const UserAlloc& ua, size_t bytes, hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  // called without the lock: the allocator may call back into anything
  void* p = ua.alloc(bytes, dev, s, ua.ctx);
  if (!p) return nullptr;
  std::lock_guard<std::mutex> lk(g_user_mu);
  g_user_live[p] = UserBlock{bytes, dev, s, ua};
  return p;
}

// true if p came from a caller-supplied allocator (and was given back)
bool user_free(void* p, hipStream_t s) {
  UserBlock ub{};
  {
    std::lock_guard<std::mutex> lk(g_user_mu);
    auto it = g_user_live.find(p);
    if (it == g_user_live.end()) return false;
    ub = it->second;
    g_user_live.erase(it);
  }
  // the allocator orders reuse after the work on the block's own stream; if
  // the last use was on another stream, wait for it here
  if (s != ub.stream) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess && hipEventRecord(ev, s) == hipSuccess)
      (void)hipEventSynchronize(ev);
    else
      (void)hipDeviceSynchronize();
    if (ev) (void)hipEventDestroy(ev);
  }
  ub.ua.free(p, ub.bytes, ub.dev, ub.stream, ub.ua.ctx);
  return true;
}
}  // namespace

void* pool_alloc(size_t bytes, hipStream_t s) {
  UserAlloc ua;
  {
    std::lock_guard<std::mutex> lk(g_user_mu);
    ua = g_user;
  }
  if (ua.alloc) return user_alloc(ua, bytes ? bytes : 1, s);
  std::call_once(g_dev_once, [] {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) g_dev_cap = tot / 4;
  });
  const size_t cls = size_class(bytes);
  void* p = nullptr;
  if (cls == 0) {
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_dev_free.find(cache_key(cls, dev));
  if (it != g_dev_free.end() && !it->second.empty()) {
    CachedBlock c = it->second.back();
    it->second.pop_back();
    g_dev_cached -= cls;
    order_after(s, c.ev);
    (void)hipEventDestroy(c.ev);
    g_dev_live[c.p] = LiveBlock{cls, dev};
    return c.p;
  }
  if (hipMallocAsync(&p, cls, s) != hipSuccess) {
    (void)hipGetLastError();
    trim_cache(dev, s);  // cached blocks of other classes go back, then try again
    if (hipMallocAsync(&p, cls, s) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  g_dev_live[p] = LiveBlock{cls, dev};
  return p;
}

void pool_free(void* p, hipStream_t s) {
  if (!p) return;
  if (user_free(p, s)) return;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_dev_live.find(p);
  if (it == g_dev_live.end()) {  // below the cached sizes
    (void)hipFreeAsync(p, s);
    return;
  }
  const LiveBlock lb = it->second;
  g_dev_live.erase(it);
  hipEvent_t ev = nullptr;
  if (g_dev_cached + lb.cls > g_dev_cap || hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ev, s) != hipSuccess) {
    if (ev) (void)hipEventDestroy(ev);
    (void)hipFreeAsync(p, s);
    return;
  }
  g_dev_free[cache_key(lb.cls, lb.dev)].push_back(CachedBlock{p, ev});
  g_dev_cached += lb.cls;
}

void* Arena::alloc(size_t bytes) {
  std::lock_guard<std::mutex> lock(mu);
  bytes = round_up(bytes ? bytes : 1, 256);
  if (bytes > left) {
    const size_t chunk = std::max(bytes, this->chunk);
    void* p = pool_alloc(chunk, stream);
    if (!p) return nullptr;
    chunks.push_back(p);
    cur = static_cast<char*>(p);
    left = chunk;
  }
  void* r = cur;
  cur += bytes;
  left -= bytes;
  total += bytes;
  return r;
}

void Arena::release() {
  for (void* p : chunks) pool_free(p, stream);
  chunks.clear();
  cur = nullptr;
  left = 0;
  total = 0;
}

void* Scratch::ensure(size_t bytes, hipStream_t s) {
  bytes = round_up(bytes ? bytes : 1, 256);
  if (bytes <= cap) {
    if (s != last && p) {  // first use on another stream: wait for the previous one
      hipEvent_t ev;
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
        if (hipEventRecord(ev, last) == hipSuccess) order_after(s, ev);
        else (void)hipStreamSynchronize(last);
        (void)hipEventDestroy(ev);
      } else {
        (void)hipStreamSynchronize(last);
      }
    }
    last = s;
    return p;
  }
  const size_t want = std::max(bytes, cap * 3 / 2);
  if (p) pool_free(p, last);
  p = nullptr;
  cap = 0;
  last = s;
  p = pool_alloc(want, s);
  if (!p) return nullptr;
  cap = want;
  return p;
}

void Scratch::release() {
  pool_free(p, last);
  p = nullptr;
  cap = 0;
}

namespace {
// Pinned host blocks of the staging buffers, kept for reuse (power-of-two
// sizes), so that handles created and destroyed in a loop do not allocate
// and free pinned memory each time.
std::mutex g_pin_mu;
std::vector<std::pair<size_t, char*>> g_pin_free;
size_t g_pin_bytes = 0;
constexpr size_t kPinKeep = (size_t)1 << 30;

char* pinned_get(size_t bytes) {
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    for (size_t q = 0; q < g_pin_free.size(); ++q)
      if (g_pin_free[q].first == bytes) {
        char* p = g_pin_free[q].second;
        g_pin_free.erase(g_pin_free.begin() + q);
        g_pin_bytes -= bytes;
        return p;
      }
  }
  char* p = nullptr;
  if (hipHostMalloc(reinterpret_cast<void**>(&p), bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
  return p;
}

void pinned_put(char* p, size_t bytes) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (g_pin_bytes + bytes <= kPinKeep) {  // every handle of a large batch holds one
      g_pin_free.emplace_back(bytes, p);
      g_pin_bytes += bytes;
      return;
    }
  }
  (void)hipHostFree(p);
}
}  // namespace

// Frees every cached device block, each once its last use has finished, and
// every kept pinned host block.  Blocks in use are not touched.  Returns the
// first runtime error; the remaining blocks are still released.
hipError_t release_cached_memory() {
  hipError_t first = hipSuccess;
  auto note = [&first](hipError_t e) {
    if (first == hipSuccess && e != hipSuccess) first = e;
  };
  {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    int cur = 0;
    note(hipGetDevice(&cur));
    std::vector<int> devs;
    for (auto& kv : g_dev_free) {
      const int dev = (int)(kv.first & 255);
      const size_t cls = (size_t)(kv.first >> 8);
      note(hipSetDevice(dev));
      for (CachedBlock& c : kv.second) {
        note(hipEventSynchronize(c.ev));
        (void)hipEventDestroy(c.ev);
        note(hipFreeAsync(c.p, nullptr));
        g_dev_cached -= cls;
      }
      if (!kv.second.empty() && std::find(devs.begin(), devs.end(), dev) == devs.end()) devs.push_back(dev);
    }
    g_dev_free.clear();
    for (int dev : devs) {  // the runtime pool gives freed memory back at a synchronization
      note(hipSetDevice(dev));
      note(hipStreamSynchronize(nullptr));
    }
    note(hipSetDevice(cur));
  }
  std::vector<std::pair<size_t, char*>> pins;
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    pins.swap(g_pin_free);
    g_pin_bytes = 0;
  }
  for (auto& b : pins) note(hipHostFree(b.second));
  return first;
}

hipError_t Staging::init(size_t bytes, hipStream_t s) {
  size_t b = (size_t)1 << 20;
  while (b < bytes) b <<= 1;
  stream = s;
  used = 0;
  stream_used = false;
  // a retired block whose readers have run, or, with too many retired
  // blocks (many stream-ordered calls queued and not yet run), the oldest
  // one once its readers have run
  constexpr size_t kMaxSpares = 32;
  for (size_t q = 0; q < spares.size(); ++q) {
    const bool last_try = spares.size() >= kMaxSpares && q == 0;
    if (spares[q].cap < b && !last_try) continue;
    const hipError_t qe = last_try ? hipEventSynchronize(spares[q].ev) : hipEventQuery(spares[q].ev);
    if (qe == hipErrorNotReady) continue;
    if (qe != hipSuccess) return qe;
    Spare sp = spares[q];
    spares.erase(spares.begin() + q);
    (void)hipEventDestroy(sp.ev);
    if (sp.cap < b) {  // too small: free it and look again
      pinned_put(sp.host, sp.cap);
      pool_free(sp.dev, s);
      --q;
      continue;
    }
    host = sp.host;
    dev = sp.dev;
    cap = sp.cap;
    return hipSuccess;
  }
  cap = b;
  host = pinned_get(b);
  if (!host) {
    cap = 0;
    return hipErrorOutOfMemory;
  }
  dev = static_cast<char*>(pool_alloc(b, s));
  if (!dev) {
    pinned_put(host, b);
    host = nullptr;
    cap = 0;
    return hipErrorOutOfMemory;
  }
  return hipSuccess;
}

hipError_t Staging::retire() {
  if (!host || used == 0) return hipSuccess;
  hipEvent_t ev = nullptr;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev, stream);
  if (e != hipSuccess) {  // cannot fence: wait instead, and keep the block
    if (ev) (void)hipEventDestroy(ev);
    e = hipStreamSynchronize(stream);
    used = 0;
    return e;
  }
  spares.push_back(Spare{host, dev, cap, ev});
  host = dev = nullptr;
  cap = used = 0;
  stream_used = false;
  return hipSuccess;
}

void Staging::release() {
  // queued copies and kernels may still read the blocks: they are reused only after them
  if (host && stream_used) (void)hipStreamSynchronize(stream);
  if (host) pinned_put(host, cap);
  if (dev) pool_free(dev, stream);
  for (Spare& sp : spares) {  // their readers have run once the event completed
    (void)hipEventSynchronize(sp.ev);
    (void)hipEventDestroy(sp.ev);
    pinned_put(sp.host, sp.cap);
    pool_free(sp.dev, nullptr);
  }
  spares.clear();
  host = dev = nullptr;
  cap = used = 0;
}

// a block of at least `need` bytes with nothing pushed yet
static bool fresh_block(Staging& st, size_t need) {
  if (st.host && st.used == 0 && need <= st.cap) return true;
  if (st.host && st.retire() != hipSuccess) return false;
  if (st.host && need <= st.cap) return true;  // retire fell back to a wait
  if (st.host) {  // too small: give it back
    if (st.stream_used && hipStreamSynchronize(st.stream) != hipSuccess) return false;
    pinned_put(st.host, st.cap);
    pool_free(st.dev, st.stream);
    st.host = st.dev = nullptr;
    st.cap = st.used = 0;
  }
  return st.init(std::max(need * 2, (size_t)1 << 20), st.stream) == hipSuccess;
}

void* Staging::push(const void* src, size_t bytes) {
  const size_t need = round_up(bytes ? bytes : 1, 256);
  if (!host || used + need > cap) {
    if (!fresh_block(*this, need)) return nullptr;
  }
  std::memcpy(host + used, src, bytes);
  stream_used = true;
  if (hipMemcpyAsync(dev + used, host + used, bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
    return nullptr;
  void* r = dev + used;
  used += need;
  return r;
}

bool Staging::reserve(std::initializer_list<size_t> sizes) {
  size_t total = 0;
  for (size_t b : sizes) total += round_up(b ? b : 1, 256);
  if (host && used + total <= cap) return true;
  return fresh_block(*this, total);
}

long long resident_bytes(const Handle& H) {
  long long b = (long long)H.gen->total / std::max<long>(1, H.gen.use_count());
  b += (long long)(H.work_id.cap + H.work_sample.cap + H.work_mv.cap + H.work_misc.cap);
  b += (long long)H.staging.cap;
  for (const Staging::Spare& sp : H.staging.spares) b += (long long)sp.cap;
  return b;
}

long long Handle::generator_bytes() const {
  long long b = 0;
  for (size_t t = 0; t < nodes.size(); ++t) {
    const Node& v = nodes[t];
    if (v.leaf()) b += (long long)v.size() * v.size() * 8;
    if (t != 0) {
      b += (long long)(v.mr - v.kr) * v.kr * 8 + (long long)(v.mc - v.kc) * v.kc * 8;
      b += (long long)(v.mr + v.mc + v.kr + v.kc) * 4;
    }
    if (!v.leaf()) {
      const Node& a = nodes[v.left];
      const Node& c = nodes[v.right];
      b += (long long)(a.kr * c.kc + c.kr * a.kc) * 8;
    }
  }
  return b;
}

}  // namespace hss

// ---------------------------------------------------------------------------
// tree
// ---------------------------------------------------------------------------
namespace {

hss_status build_tree(Handle& H, long long n, const hss_tree* tree, int leaf_size) {
  std::vector<Node>& nd = H.nodes;
  nd.clear();
  if (!tree) {
    if (leaf_size < 1) return fail(HSS_ERR_ARG, "leaf_size must be >= 1");
    Node r;
    r.lo = 0;
    r.hi = (int)n;
    nd.push_back(r);
    for (size_t head = 0; head < nd.size(); ++head) {  // breadth-first
      const int lo = nd[head].lo, hi = nd[head].hi, m = hi - lo;
      if (m > leaf_size) {
        const int mid = lo + m / 2;
        Node a, b;
        a.lo = lo;
        a.hi = mid;
        a.parent = (int)head;
        b.lo = mid;
        b.hi = hi;
        b.parent = (int)head;
        nd.push_back(a);
        nd.push_back(b);
        nd[head].left = (int)nd.size() - 2;
        nd[head].right = (int)nd.size() - 1;
      }
    }
  } else {
    const int nn = tree->n_nodes;
    if (nn < 1 || !tree->lo || !tree->hi || !tree->left || !tree->right)
      return fail(HSS_ERR_ARG, "tree arrays missing");
    nd.resize(nn);
    for (int t = 0; t < nn; ++t) {
      nd[t].lo = tree->lo[t];
      nd[t].hi = tree->hi[t];
      nd[t].left = tree->left[t];
      nd[t].right = tree->right[t];
    }
    if (nd[0].lo != 0 || nd[0].hi != n) return fail(HSS_ERR_ARG, "root interval must be [0, n)");
    std::vector<int> seen(nn, 0);
    seen[0] = 1;
    for (int t = 0; t < nn; ++t) {
      Node& v = nd[t];
      if (v.hi <= v.lo) return fail(HSS_ERR_ARG, "empty tree interval");
      if ((v.left < 0) != (v.right < 0)) return fail(HSS_ERR_ARG, "node with one child");
      if (v.left >= 0) {
        if (v.left >= nn || v.right >= nn || v.left == 0 || v.right == 0)
          return fail(HSS_ERR_ARG, "bad child index");
        Node &a = nd[v.left], &b = nd[v.right];
        if (a.lo != v.lo || a.hi != b.lo || b.hi != v.hi)
          return fail(HSS_ERR_ARG, "children do not split the parent interval");
        if (seen[v.left]++ || seen[v.right]++) return fail(HSS_ERR_ARG, "node reached twice");
        a.parent = t;
        b.parent = t;
      }
    }
    for (int t = 0; t < nn; ++t)
      if (!seen[t]) return fail(HSS_ERR_ARG, "node not reachable from the root");
  }
  // heights (children before parents: iterate until stable; depth-first order)
  std::vector<int> order;
  order.reserve(nd.size());
  std::vector<int> st{0};
  while (!st.empty()) {
    int t = st.back();
    st.pop_back();
    order.push_back(t);
    if (nd[t].left >= 0) {
      st.push_back(nd[t].left);
      st.push_back(nd[t].right);
    }
  }
  for (auto it = order.rbegin(); it != order.rend(); ++it) {
    Node& v = nd[*it];
    v.height = v.leaf() ? 0 : 1 + std::max(nd[v.left].height, nd[v.right].height);
  }
  H.height = nd[0].height;
  H.levels.assign(H.height, {});
  for (size_t t = 1; t < nd.size(); ++t) H.levels[nd[t].height].push_back((int)t);
  H.leaves.clear();
  for (size_t t = 0; t < nd.size(); ++t)
    if (nd[t].leaf()) H.leaves.push_back((int)t);
  std::sort(H.leaves.begin(), H.leaves.end(),
            [&](int a, int b) { return nd[a].lo < nd[b].lo; });
  return HSS_OK;
}

// generators: kept with the handle
template <typename T>
T* arena_alloc(Handle& H, size_t count) {
  return static_cast<T*>(H.gen->alloc(count * sizeof(T)));
}
// compression-only buffers (global R and S, local samples, R_tau): freed
// when the compression returns
template <typename T>
T* work_alloc(Arena& W, size_t count) {
  return static_cast<T*>(W.alloc(count * sizeof(T)));
}

// ---------------------------------------------------------------------------
// compression
// ---------------------------------------------------------------------------
struct EventTimer {  // HIP events on the compression stream, summed at the end
  std::vector<hipEvent_t> ev;
  // begin, end, category (0 sample, 1 levels, 2 id, 3 sample GEMM, 4 level GEMMs, 5 gathers)
  std::vector<int> b, e, cat;
  hipStream_t s = nullptr;
  int begin() {  // an event that cannot be made or recorded is kept as null and not timed
    hipEvent_t x = nullptr;
    if (hipEventCreate(&x) != hipSuccess) {
      x = nullptr;
    } else if (hipEventRecord(x, s) != hipSuccess) {
      (void)hipEventDestroy(x);
      x = nullptr;
    }
    ev.push_back(x);
    return (int)ev.size() - 1;
  }
  void end(int bi, int c) {
    const int ei = begin();
    b.push_back(bi);
    e.push_back(ei);
    cat.push_back(c);
  }
  void finish(double* acc) {
    (void)hipStreamSynchronize(s);
    for (size_t i = 0; i < b.size(); ++i) {
      float ms = 0;
      if (ev[b[i]] && ev[e[i]] && hipEventElapsedTime(&ms, ev[b[i]], ev[e[i]]) == hipSuccess) acc[cat[i]] += ms;
    }
    for (auto x : ev)
      if (x) (void)hipEventDestroy(x);
    ev.clear();
    b.clear();
    e.clear();
    cat.clear();
  }
};

// New sample columns for several matrices: columns c0..c1-1 of R^r, R^c and
// of S^r, S^c of each, on the lead handle's stream and sampling workspace.
struct SampleReq {
  Handle* H;
  const void* A;
  long long lda;
  int c0, c1;
};

hss_status sample_batch(Handle& L, const std::vector<SampleReq>& reqs, EventTimer& tm) {
  if (reqs.empty()) return HSS_OK;
  const int ev0 = tm.begin();
  const int prec = L.opts.sample_prec;
  // the new random columns of every matrix and side in one launch, rounded
  // to the products' precision (used as such from here on)
  std::vector<RngJob> rj;
  for (const SampleReq& q : reqs) {
    Handle& H = *q.H;
    const int c0 = q.c0, c1 = q.c1, nc = c1 - c0;
    if (nc <= 0) continue;
    if (H.opts.R_user_r) {
      HIPCHK(hipMemcpy2DAsync(H.Rr + c0, H.ldg * 8, H.opts.R_user_r + c0, H.opts.ld_R_user * 8,
                              (size_t)nc * 8, H.n, hipMemcpyDeviceToDevice, L.stream));
      HIPCHK(hipMemcpy2DAsync(H.Rc + c0, H.ldg * 8, H.opts.R_user_c + c0, H.opts.ld_R_user * 8,
                              (size_t)nc * 8, H.n, hipMemcpyDeviceToDevice, L.stream));
      if (prec != HSS_SAMPLE_F64) {
        launch_round_r(H.Rr, H.ldg, H.n, c0, c1, prec, L.stream);
        launch_round_r(H.Rc, H.ldg, H.n, c0, c1, prec, L.stream);
      }
    } else {
      rj.push_back(RngJob{H.opts.seed, 0, H.n, c0, nc, H.Rr + c0, H.ldg});
      rj.push_back(RngJob{H.opts.seed, 1, H.n, c0, nc, H.Rc + c0, H.ldg});
    }
  }
  HIPCHK(launch_random_normal_batched(rj.data(), (int)rj.size(), prec, L.staging, L.stream));
  const int evg = tm.begin();
  if (prec != HSS_SAMPLE_F64 && reqs.size() > 1) {  // all matrices in one launch per side
    std::vector<SampleJob> jobs;
    for (const SampleReq& q : reqs) {
      const Handle& H = *q.H;
      if (q.c1 <= q.c0) continue;
      SampleJob j{};
      j.A = static_cast<const float*>(q.A);
      j.lda = q.lda;
      j.n = H.n;
      j.leaf_of = H.leaf_of;
      j.ncols = q.c1 - q.c0;
      j.Rr = H.Rr + q.c0;
      j.Rc = H.Rc + q.c0;
      j.ldr = H.ldg;
      j.Sr = H.Sr + q.c0;
      j.Sc = H.Sc + q.c0;
      j.lds = H.ldg;
      jobs.push_back(j);
    }
    const long long wd = sample_mixed_grouped_workspace_doubles(jobs.data(), (int)jobs.size());
    double* work = static_cast<double*>(L.work_sample.ensure((size_t)std::max(1LL, wd) * 8, L.stream));
    if (!work) return fail(HSS_ERR_ALLOC, "sampling workspace");
    HIPCHK(launch_sample_mixed_grouped(jobs.data(), (int)jobs.size(), prec, work, L.staging, L.stream));
    L.n_sgemm += 2;
  } else {
    for (const SampleReq& q : reqs) {
      const Handle& H = *q.H;
      const int c0 = q.c0, nc = q.c1 - q.c0;
      if (nc <= 0) continue;
      const long long wd = prec == HSS_SAMPLE_F64 ? sample_workspace_doubles(H.n, nc)
                                                  : sample_mixed_workspace_doubles(H.n, nc);
      double* work = nullptr;
      if (wd > 0) {
        work = static_cast<double*>(L.work_sample.ensure((size_t)wd * 8, L.stream));
        if (!work) return fail(HSS_ERR_ALLOC, "sampling workspace");
      }
      if (prec == HSS_SAMPLE_F64)
        launch_sample(q.A, H.dtype, H.n, q.lda, H.leaf_of, nc, H.Rr + c0, H.Rc + c0, H.ldg, H.Sr + c0,
                      H.Sc + c0, H.ldg, work, L.stream);
      else
        HIPCHK(launch_sample_mixed(static_cast<const float*>(q.A), H.n, q.lda, H.leaf_of, nc, prec,
                                   H.Rr + c0, H.Rc + c0, H.ldg, H.Sr + c0, H.Sc + c0, H.ldg, work,
                                   L.stream));
      HIPCHK(hipGetLastError());
      L.n_sgemm += 2;
    }
  }
  tm.end(evg, 3);
  tm.end(ev0, 0);
  // each product 2 n^2 nc flops; bytes: A once per product, R read, S written
  for (const SampleReq& q : reqs) {
    const Handle& H = *q.H;
    const int nc = q.c1 - q.c0;
    L.sgemm_flops += 4.0 * (double)H.n * (double)H.n * nc;
    L.sgemm_bytes += 2.0 * ((double)H.n * (double)H.n * (H.dtype == HSS_F32 ? 4 : 8) +
                            2.0 * (double)H.n * nc * 8);
  }
  return HSS_OK;
}

// Source rows of the "R_in" stack of node t: R(I_t) at a leaf, [R_a; R_b] above.
Seg r_in(const Handle& H, int t, bool row_side, int c0) {
  const Node& v = H.nodes[t];
  Seg s{};
  s.ld = H.ldg;
  s.split = INT_MAX;
  if (v.leaf()) {
    s.p0 = (row_side ? H.Rr : H.Rc) + (long long)v.lo * H.ldg + c0;
  } else {
    const Node& a = H.nodes[v.left];
    const Node& b = H.nodes[v.right];
    s.p0 = (row_side ? a.Rr : a.Rc) + c0;
    s.p1 = (row_side ? b.Rr : b.Rc) + c0;
    s.split = row_side ? a.kc : a.kr;
  }
  return s;
}

// Algorithmic bytes of a batched GEMM launch: A, B and D once, C when read.
double gemm_bytes(const std::vector<GemmDesc>& gd) {
  double b = 0.0;
  for (const GemmDesc& g : gd)
    b += 8.0 * ((double)g.M * g.K + (double)g.K * g.N + (double)g.M * g.N * (g.beta != 0.0 ? 2.0 : 1.0));
  return b;
}

// Algorithmic bytes of a gather launch: each entry read from A, written in FP64.
double gather_bytes_of(const std::vector<GatherDesc>& g, int dtype) {
  double b = 0.0;
  for (const GatherDesc& d : g) b += (double)d.nr * d.nc * ((dtype == HSS_F32 ? 4.0 : 8.0) + 8.0);
  return b;
}

// One node of one matrix in a level batch: node t of handle H, whose matrix
// has d sample columns so far; `forced` accepts every ID (d_max reached).
struct Item {
  Handle* H;
  const void* A;
  long long lda;
  int t;
  int d;
  bool forced;
  char* any_fail;  // set when an ID of this node fails the rule
};

// The level step of Alg. 1 / Alg. 5 for a batch of nodes that may belong to
// different matrices: every phase is one batched launch over all of them.
// L (the lead handle) provides the stream, staging buffer, ID workspace and
// rank readback; all handles of a batch share L's stream.
hss_status process_items(Handle& L, Arena& W, std::vector<Item>& items, EventTimer& tm) {
  if (items.empty()) return HSS_OK;
  const int ev_level = tm.begin();
  auto node = [](const Item& it) -> Node& { return it.H->nodes[it.t]; };

  // (1) first visit: sizes, buffers, D or B
  std::vector<GatherDesc> gath;
  for (Item& it : items) {
    Handle& H = *it.H;
    std::vector<Node>& nd = H.nodes;
    Node& v = nd[it.t];
    if (v.set_up) continue;
    if (v.leaf()) {
      const int m = v.size();
      v.mr = v.mc = m;
      v.Sr = H.Sr + (long long)v.lo * H.ldg;
      v.Sc = H.Sc + (long long)v.lo * H.ldg;
      v.D = arena_alloc<double>(H, (size_t)m * m);
      if (!v.D) return fail(HSS_ERR_ALLOC, "leaf D");
      GatherDesc g{};
      g.nr = g.nc = m;
      g.out = v.D;
      g.ldo = m;
      g.row_off = g.col_off = v.lo;
      g.A = it.A;
      g.lda = it.lda;
      gath.push_back(g);
    } else {
      const Node& a = nd[v.left];
      const Node& b = nd[v.right];
      v.mr = a.kr + b.kr;
      v.mc = a.kc + b.kc;
      v.B12 = arena_alloc<double>(H, (size_t)a.kr * b.kc);
      v.B21 = arena_alloc<double>(H, (size_t)b.kr * a.kc);
      v.Sr = work_alloc<double>(W, (size_t)v.mr * H.ldg);
      v.Sc = work_alloc<double>(W, (size_t)v.mc * H.ldg);
      if (!v.B12 || !v.B21 || !v.Sr || !v.Sc) return fail(HSS_ERR_ALLOC, "inner node buffers");
      GatherDesc g{};
      g.A = it.A;
      g.lda = it.lda;
      g.rows = a.Ir;
      g.cols = b.Ic;
      g.nr = a.kr;
      g.nc = b.kc;
      g.out = v.B12;
      g.ldo = b.kc;
      gath.push_back(g);
      g.rows = b.Ir;
      g.cols = a.Ic;
      g.nr = b.kr;
      g.nc = a.kc;
      g.out = v.B21;
      g.ldo = a.kc;
      gath.push_back(g);
    }
    v.perm_r = arena_alloc<int>(H, (size_t)v.mr);
    v.perm_c = arena_alloc<int>(H, (size_t)v.mc);
    v.Er = arena_alloc<double>(H, (size_t)v.mr * v.mr / 4 + 1);
    v.Ec = arena_alloc<double>(H, (size_t)v.mc * v.mc / 4 + 1);
    if (!v.perm_r || !v.perm_c || !v.Er || !v.Ec) return fail(HSS_ERR_ALLOC, "ID buffers");
    v.cdone = 0;
    v.set_up = true;
  }
  const int ev_g = tm.begin();
  HIPCHK(launch_gather(items[0].A, L.dtype, items[0].lda, gath.data(), (int)gath.size(), L.staging,
                       L.stream));
  tm.end(ev_g, 5);
  L.gather_bytes += gather_bytes_of(gath, L.dtype);

  // (2) local samples of inner nodes, columns [cdone, d) (Alg. 1 / Alg. 5)
  std::vector<GemmDesc> gd;
  for (Item& it : items) {
    Handle& H = *it.H;
    std::vector<Node>& nd = H.nodes;
    Node& v = nd[it.t];
    const int d = it.d;
    if (v.leaf() || v.cdone >= d) continue;
    const Node& a = nd[v.left];
    const Node& b = nd[v.right];
    const int c0 = v.cdone, N = d - c0;
    auto mk = [&](int M, int K, const double* Am, long long lda_, int tr, const double* Bp,
                  const double* Cp, const int* cmap, double* Dp) {
      GemmDesc g{};
      g.M = M;
      g.N = N;
      g.K = K;
      g.A = Am;
      g.lda = lda_;
      g.transA = tr;
      g.B = Seg{Bp, nullptr, H.ldg, INT_MAX, nullptr};
      g.C = Seg{Cp, nullptr, H.ldg, INT_MAX, cmap};
      g.D = SegOut{Dp, nullptr, H.ldg, INT_MAX, nullptr};
      g.alpha = -1.0;
      g.beta = 1.0;
      gd.push_back(g);
    };
    // S^r_loc = [S^r_a - B_ab R^r_b ; S^r_b - B_ba R^r_a]
    mk(a.kr, b.kc, v.B12, b.kc, 0, b.Rr + c0, a.Sr + c0, a.perm_r, v.Sr + c0);
    mk(b.kr, a.kc, v.B21, a.kc, 0, a.Rr + c0, b.Sr + c0, b.perm_r, v.Sr + (long long)a.kr * H.ldg + c0);
    // S^c_loc = [S^c_a - B_ba^T R^c_b ; S^c_b - B_ab^T R^c_a]
    mk(a.kc, b.kr, v.B21, a.kc, 1, b.Rc + c0, a.Sc + c0, a.perm_c, v.Sc + c0);
    mk(b.kc, a.kr, v.B12, b.kc, 1, a.Rc + c0, b.Sc + c0, b.perm_c, v.Sc + (long long)a.kc * H.ldg + c0);
  }
  const int ev_g1 = tm.begin();
  HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), L.staging, L.stream));
  tm.end(ev_g1, 4);
  L.lgemm_bytes += gemm_bytes(gd);

  // (3) interpolative decompositions of the nodes not yet compressed
  std::vector<int> idn;  // indices into items
  for (size_t q = 0; q < items.size(); ++q)
    if (node(items[q]).state != HSS_COMPRESSED) idn.push_back((int)q);
  std::vector<char> passed(items.size(), 0);
  if (!idn.empty()) {
    const int np = 2 * (int)idn.size();
    std::vector<IdProblem> pr(np);
    for (int q = 0; q < np; ++q) {
      const Item& it = items[idn[q / 2]];
      const Node& v = node(it);
      const bool rs = (q % 2) == 0;
      IdProblem& p = pr[q];
      p.Y = rs ? v.Sr : v.Sc;
      p.ldy = it.H->ldg;
      p.m = rs ? v.mr : v.mc;
      p.d = it.d;
      p.perm = rs ? v.perm_r : v.perm_c;
      p.E = rs ? v.Er : v.Ec;
      const int pm = it.H->opts.p_margin;
      p.kfail = (it.forced || it.d - pm < 0) ? -1 : it.d - pm;
      p.partner = rs ? q + 1 : q - 1;  // the node fails if either side does (Sec. 3.3)
    }
    const size_t wb = id_workspace_bytes(pr.data(), np);
    void* wk = L.work_id.ensure(wb, L.stream);
    if (!wk) return fail(HSS_ERR_ALLOC, "ID workspace");
    if (L.k_host_cap < np) {
      if (L.k_host) (void)hipHostFree(L.k_host);
      L.k_host = nullptr;
      HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&L.k_host), (size_t)np * 2 * 4, hipHostMallocDefault));
      L.k_host_cap = np * 2;
    }
    const int ev_id = tm.begin();
    const double t_id0 = L.verbose >= 2 ? now_ms() : 0.0;
    HIPCHK(launch_id_factor(pr.data(), np, L.opts.rtol, wk, L.work_id.cap, L.k_host, L.staging,
                            L.stream));
    if (L.verbose >= 2) {  // the factor call has read the ranks back: its work is done
      int hmin = INT_MAX, hmax = 0, nfail = 0, mmax = 0;
      for (size_t q = 0; q < idn.size(); ++q) {
        const Item& it = items[idn[q]];
        const Node& v = node(it);
        hmin = std::min(hmin, v.height);
        hmax = std::max(hmax, v.height);
        mmax = std::max(mmax, std::max(v.mr, v.mc));
        const int kf = it.d - it.H->opts.p_margin;
        const int kr = L.k_host[2 * q], kc = L.k_host[2 * q + 1];
        if (!it.forced && ((kr > kf && kr < v.mr) || (kc > kf && kc < v.mc))) ++nfail;
      }
      std::fprintf(stderr, "[hss] level h=%d..%d d=%d: %zu ID nodes (%d fail), max m %d: %.2f ms\n", hmin, hmax,
                   items[0].d, idn.size(), nfail, mmax, now_ms() - t_id0);
      std::fflush(stderr);
    }
    L.staging.reset();
    for (int q = 0; q < np; ++q)  // Householder QR of d x m to k steps: about 4 d m k flops
      L.id_flops += 4.0 * (double)pr[q].d * (double)pr[q].m * (double)L.k_host[q];
    std::vector<int> sel;
    for (size_t q = 0; q < idn.size(); ++q) {
      Item& it = items[idn[q]];
      Handle& H = *it.H;
      Node& v = node(it);
      const int kf = it.d - H.opts.p_margin;
      const int kr = L.k_host[2 * q], kc = L.k_host[2 * q + 1];
      const bool fr = (kr > kf && kr < v.mr), fc = (kc > kf && kc < v.mc);
      if (!it.forced && (fr || fc)) {
        v.state = HSS_PARTIALLY_COMPRESSED;
        *it.any_fail = 1;
        continue;
      }
      v.kr = kr;
      v.kc = kc;
      v.Rr = work_alloc<double>(W, (size_t)kc * H.ldg);
      v.Rc = work_alloc<double>(W, (size_t)kr * H.ldg);
      v.Ir = arena_alloc<int>(H, (size_t)kr);
      v.Ic = arena_alloc<int>(H, (size_t)kc);
      if (!v.Rr || !v.Rc || !v.Ir || !v.Ic) return fail(HSS_ERR_ALLOC, "node R / index buffers");
      v.state = HSS_COMPRESSED;
      passed[idn[q]] = 1;
      sel.push_back(2 * (int)q);
      sel.push_back(2 * (int)q + 1);
    }
    HIPCHK(launch_id_finish(pr.data(), np, L.k_host, sel.data(), (int)sel.size(), wk, L.staging,
                            L.stream));
    tm.end(ev_id, 2);
  }

  // (4) skeleton index sets of the nodes compressed now: I_tau = I_in(J)
  std::vector<IndexDesc> ix;
  for (size_t q = 0; q < items.size(); ++q) {
    if (!passed[q]) continue;
    const std::vector<Node>& nd = items[q].H->nodes;
    const Node& v = nd[items[q].t];
    IndexDesc a{}, c{};
    a.perm = v.perm_r;
    a.k = v.kr;
    c.perm = v.perm_c;
    c.k = v.kc;
    if (v.leaf()) {
      a.split = c.split = INT_MAX;
      a.off0 = c.off0 = v.lo;
    } else {
      const Node& l = nd[v.left];
      const Node& r = nd[v.right];
      a.b0 = l.Ir;
      a.b1 = r.Ir;
      a.split = l.kr;
      c.b0 = l.Ic;
      c.b1 = r.Ic;
      c.split = l.kc;
    }
    a.out = v.Ir;
    c.out = v.Ic;
    if (a.k > 0) ix.push_back(a);
    if (c.k > 0) ix.push_back(c);
  }
  HIPCHK(launch_index_compose(ix.data(), (int)ix.size(), L.staging, L.stream));

  // (5) R^r_tau = V^T R^r_in and R^c_tau = U^T R^c_in on the new columns
  gd.clear();
  for (size_t q = 0; q < items.size(); ++q) {
    const Item& it = items[q];
    const Handle& H = *it.H;
    Node& v = node(it);
    if (v.state != HSS_COMPRESSED) continue;
    const int d = it.d;
    const int c0 = passed[q] ? 0 : v.cdone;
    if (c0 >= d) continue;
    for (int side = 0; side < 2; ++side) {
      // side 0: R^r_tau uses V (perm_c, Ec, kc, mc); side 1: R^c_tau uses U
      const int k = side == 0 ? v.kc : v.kr;
      const int m = side == 0 ? v.mc : v.mr;
      const int* perm = side == 0 ? v.perm_c : v.perm_r;
      Seg src = r_in(H, it.t, side == 0, c0);
      GemmDesc g{};
      g.M = k;
      g.N = d - c0;
      g.K = m - k;
      g.A = side == 0 ? v.Ec : v.Er;
      g.lda = k;
      g.transA = 1;
      g.B = src;
      g.B.map = perm + k;
      g.C = src;
      g.C.map = perm;
      g.D = SegOut{(side == 0 ? v.Rr : v.Rc) + c0, nullptr, H.ldg, INT_MAX, nullptr};
      g.alpha = 1.0;
      g.beta = 1.0;
      gd.push_back(g);
    }
  }
  const int ev_g2 = tm.begin();
  HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), L.staging, L.stream));
  tm.end(ev_g2, 4);
  L.lgemm_bytes += gemm_bytes(gd);
  for (Item& it : items) node(it).cdone = it.d;
  tm.end(ev_level, 1);
  // no wait here: the next level's ID readback orders the host after this
  // level, and the staging block is only reused once its readers have run
  return HSS_OK;
}

// One matrix of a compression batch.
struct Job {
  Handle* H;
  const void* A;
  long long lda;
  int d = 0;
  bool forced = false;
  bool done = false;
  std::vector<char> ext;
};

// Adaptive randomized compression (Alg. 1 with the late-notification
// schedule of Alg. 5, level-synchronous) of every matrix of the batch
// together: a pass visits the heights 0, 1, ... and each height is one
// level batch over the unfinished matrices; a matrix that still has failed
// nodes after a pass draws dd more random columns; the passes go on until
// every matrix is done.  jobs[0].H is the lead handle.
hss_status compress_batch(std::vector<Job>& jobs) {
  const double t0 = now_ms();
  Handle& L = *jobs[0].H;
  EventTimer tm;
  tm.s = L.stream;
  Arena W;  // compression-only buffers of the whole batch
  W.chunk = (size_t)256 << 20;
  W.stream = L.stream;
  std::vector<GatherDesc> single;
  std::vector<SampleReq> first;
  int maxh = 0;
  for (Job& j : jobs) {
    Handle& H = *j.H;
    std::vector<Node>& nd = H.nodes;
    const long long n = H.n;
    if (nd[0].leaf()) {  // a single leaf: D = A
      Node& r = nd[0];
      r.D = arena_alloc<double>(H, (size_t)n * n);
      if (!r.D) return fail(HSS_ERR_ALLOC, "D");
      GatherDesc g{};
      g.nr = g.nc = (int)n;
      g.out = r.D;
      g.ldo = n;
      g.A = j.A;
      g.lda = j.lda;
      single.push_back(g);
      j.done = true;
      continue;
    }
    const int dmax = H.opts.d_max;
    H.ldg = (long long)round_up((size_t)dmax, 8);
    H.Rr = work_alloc<double>(W, (size_t)n * H.ldg);
    H.Rc = work_alloc<double>(W, (size_t)n * H.ldg);
    H.Sr = work_alloc<double>(W, (size_t)n * H.ldg);
    H.Sc = work_alloc<double>(W, (size_t)n * H.ldg);
    H.leaf_of = work_alloc<int>(W, (size_t)n);
    if (!H.Rr || !H.Rc || !H.Sr || !H.Sc || !H.leaf_of)
      return fail(HSS_ERR_ALLOC, "random matrices / samples (n x d_max doubles each)");
    const int nl = (int)H.leaves.size();
    std::vector<int> lo(nl), hi(nl);
    for (int q = 0; q < nl; ++q) {
      lo[q] = nd[H.leaves[q]].lo;
      hi[q] = nd[H.leaves[q]].hi;
    }
    if (!L.staging.reserve({lo.size() * 4, hi.size() * 4})) return fail(HSS_ERR_HIP, "staging");
    int* dlo = static_cast<int*>(L.staging.push(lo.data(), lo.size() * 4));
    int* dhi = static_cast<int*>(L.staging.push(hi.data(), hi.size() * 4));
    if (!dlo || !dhi) return fail(HSS_ERR_HIP, "staging");
    launch_leaf_of(nl, dlo, dhi, H.leaf_of, L.stream);
    HIPCHK(hipGetLastError());
    j.d = std::min(H.opts.d0, dmax);
    first.push_back(SampleReq{&H, j.A, j.lda, 0, j.d});
    H.passes = 0;
    H.converged = true;
    j.ext.assign(nd.size(), 0);
    maxh = std::max(maxh, H.height);
  }
  if (!single.empty())
    HIPCHK(launch_gather(single[0].A, L.dtype, single[0].lda, single.data(), (int)single.size(),
                         L.staging, L.stream));
  CHK(sample_batch(L, first, tm));
  int pass = 0;
  while (true) {
    std::vector<Job*> act;
    for (Job& j : jobs)
      if (!j.done) act.push_back(&j);
    if (act.empty()) break;
    ++pass;
    std::vector<char> fail_of(jobs.size(), 0);
    for (Job* j : act) {
      Handle& H = *j->H;
      std::vector<Node>& nd = H.nodes;
      ++H.passes;
      // a compressed node extends its samples iff a non-root ancestor is
      // unfinished (only then does anyone read the new columns)
      for (size_t t = 1; t < nd.size(); ++t) j->ext[t] = 0;
      for (int h = H.height - 1; h >= 0; --h)
        for (int t : H.levels[h]) {
          const int p = nd[t].parent;
          j->ext[t] = (p != 0) && (nd[p].state != HSS_COMPRESSED || j->ext[p]);
        }
    }
    for (int h = 0; h < maxh; ++h) {
      std::vector<Item> items;
      for (Job* j : act) {
        Handle& H = *j->H;
        if (h >= H.height) continue;
        std::vector<Node>& nd = H.nodes;
        char* af = &fail_of[j - jobs.data()];
        for (int t : H.levels[h]) {
          const Node& v = nd[t];
          if (!v.leaf() && !(nd[v.left].state == HSS_COMPRESSED && nd[v.right].state == HSS_COMPRESSED))
            continue;
          if (v.state == HSS_COMPRESSED && !j->ext[t]) continue;
          if (v.state == HSS_COMPRESSED && v.cdone >= j->d) continue;
          items.push_back(Item{&H, j->A, j->lda, t, j->d, j->forced, af});
        }
      }
      CHK(process_items(L, W, items, tm));
    }
    std::vector<SampleReq> grow;
    for (Job* j : act) {
      Handle& H = *j->H;
      const std::vector<Node>& nd = H.nodes;
      bool done = true;
      int ncomp = 0, nmax = 0;
      for (size_t t = 1; t < nd.size(); ++t) {
        if (nd[t].state != HSS_COMPRESSED) done = false;
        else ++ncomp;
        nmax = std::max(nmax, std::max(nd[t].kr, nd[t].kc));
      }
      if (L.verbose && jobs.size() == 1) {
        std::fprintf(stderr, "[hss] pass %d d=%d compressed %d/%d max rank %d (%.1f ms)\n", H.passes,
                     j->d, ncomp, (int)nd.size() - 1, nmax, now_ms() - t0);
        std::fflush(stderr);
      }
      if (done) {
        j->done = true;
        continue;
      }
      if (j->d >= H.opts.d_max) {
        j->forced = true;
        H.converged = false;
        continue;
      }
      const int dn = std::min(j->d + H.opts.dd, H.opts.d_max);
      grow.push_back(SampleReq{&H, j->A, j->lda, j->d, dn});
      j->d = dn;
    }
    CHK(sample_batch(L, grow, tm));
    if (L.verbose && jobs.size() > 1) {
      int left = 0;
      for (Job& j : jobs) left += j.done ? 0 : 1;
      std::fprintf(stderr, "[hss] batch pass %d: %d of %d matrices unfinished (%.1f ms)\n", pass, left,
                   (int)jobs.size(), now_ms() - t0);
      std::fflush(stderr);
    }
  }
  // roots: B_ab = A(I^r_a, I^c_b), B_ba = A(I^r_b, I^c_a)
  std::vector<GatherDesc> rg;
  for (Job& j : jobs) {
    Handle& H = *j.H;
    std::vector<Node>& nd = H.nodes;
    if (nd[0].leaf()) continue;
    Node& r = nd[0];
    const Node& a = nd[r.left];
    const Node& b = nd[r.right];
    r.mr = a.kr + b.kr;
    r.mc = a.kc + b.kc;
    r.B12 = arena_alloc<double>(H, (size_t)a.kr * b.kc);
    r.B21 = arena_alloc<double>(H, (size_t)b.kr * a.kc);
    if (!r.B12 || !r.B21) return fail(HSS_ERR_ALLOC, "root B");
    GatherDesc g{};
    g.A = j.A;
    g.lda = j.lda;
    g.rows = a.Ir;
    g.cols = b.Ic;
    g.nr = a.kr;
    g.nc = b.kc;
    g.out = r.B12;
    g.ldo = b.kc;
    rg.push_back(g);
    g.rows = b.Ir;
    g.cols = a.Ic;
    g.nr = b.kr;
    g.nc = a.kc;
    g.out = r.B21;
    g.ldo = a.kc;
    rg.push_back(g);
  }
  if (!rg.empty())
    HIPCHK(launch_gather(rg[0].A, L.dtype, rg[0].lda, rg.data(), (int)rg.size(), L.staging, L.stream));
  double acc[6] = {0, 0, 0, 0, 0, 0};
  tm.finish(acc);
  HIPCHK(hipStreamSynchronize(L.stream));
  L.staging.reset();
  W.release();  // the handles keep only their generators
  L.work_id.release();  // compression-only workspaces (back to the pool or cache)
  L.work_sample.release();
  for (Job& j : jobs) {
    Handle& H = *j.H;
    H.Rr = H.Rc = H.Sr = H.Sc = nullptr;
    H.leaf_of = nullptr;
    for (Node& v : H.nodes) v.Sr = v.Sc = v.Rr = v.Rc = nullptr;
  }
  const double total = now_ms() - t0;
  for (Job& j : jobs) {  // timings are those of the whole batch
    Handle& H = *j.H;
    H.d = j.d;
    H.t_sgemm = acc[3];
    H.t_sample = acc[0];
    H.t_levels = acc[1];
    H.t_id = acc[2];
    H.t_lgemm = acc[4];
    H.t_gather = acc[5];
    H.id_flops = L.id_flops;
    H.lgemm_bytes = L.lgemm_bytes;
    H.gather_bytes = L.gather_bytes;
    H.t_total = total;
    H.n_sgemm = L.n_sgemm;
    H.sgemm_flops = L.sgemm_flops;
    H.sgemm_bytes = L.sgemm_bytes;
    H.compressed = true;
  }
  return HSS_OK;
}

hss_status compress_impl(Handle& H, const void* A, long long lda) {
  std::vector<Job> jobs(1);
  jobs[0].H = &H;
  jobs[0].A = A;
  jobs[0].lda = lda;
  CHK(compress_batch(jobs));
  return H.converged ? HSS_OK : HSS_NOT_CONVERGED;
}

hss_status new_handle(hss_handle* out, long long n, hipStream_t s, hss_handle_s** hp) {
  hss_handle_s* p = new (std::nothrow) hss_handle_s();
  if (!p) return fail(HSS_ERR_ALLOC, "handle");
  p->h.n = n;
  p->h.stream = s;
  p->h.gen->stream = s;
  // generator arena chunks sized to the matrix
  p->h.gen->chunk = std::min<size_t>((size_t)64 << 20, std::max<size_t>((size_t)1 << 20, (size_t)n * 4096));
  // descriptor staging is allocated on first use
  p->h.staging.stream = s;
  *hp = p;
  (void)out;
  return HSS_OK;
}

void free_handle(hss_handle_s* p) {
  if (!p) return;
  Handle& H = p->h;
  if (H.stream) (void)hipStreamSynchronize(H.stream);
  if (H.queued) {  // stream-ordered calls still reading the generators
    (void)hipEventSynchronize(H.queued);
    (void)hipEventDestroy(H.queued);
    H.queued = nullptr;
  }
  H.gen.reset();  // frees the arena unless other handles of its batch still hold it
  H.work_id.release();
  H.work_sample.release();
  H.work_mv.release();
  H.work_misc.release();
  H.staging.release();
  if (H.k_host) (void)hipHostFree(H.k_host);
  delete p;
}

}  // namespace

// ---------------------------------------------------------------------------
// matvec (Alg. 2)
// ---------------------------------------------------------------------------
namespace hss {

hss_status sample_args(const void* A, int dtype, int sample_prec, long long n, long long lda, int ncols,
                       const double* Rr, const double* Rc, long long ldr, double* Sr, double* Sc,
                       long long lds, long long* work_doubles) {
  if (!A || n < 1 || lda < n || ncols < 0 || ldr < ncols || lds < ncols)
    return fail(HSS_ERR_ARG, "sample arguments");
  if ((Sr == nullptr) != (Rr == nullptr) || (Sc == nullptr) != (Rc == nullptr))
    return fail(HSS_ERR_ARG, "S and R must be given together");
  if (dtype != HSS_F64 && dtype != HSS_F32) return fail(HSS_ERR_ARG, "dtype");
  if (sample_prec < HSS_SAMPLE_F64 || sample_prec > HSS_SAMPLE_BF16X3)
    return fail(HSS_ERR_ARG, "unknown sample precision");
  if (sample_prec != HSS_SAMPLE_F64 && dtype != HSS_F32)
    return fail(HSS_ERR_ARG, "reduced-precision sampling needs A stored in FP32");
  *work_doubles = sample_prec == HSS_SAMPLE_F64 ? sample_workspace_doubles(n, ncols)
                                                : sample_mixed_workspace_doubles(n, ncols);
  return HSS_OK;
}

hipError_t sample_queue(const void* A, int dtype, int sample_prec, long long n, long long lda,
                        const int* leaf_of, int ncols, const double* Rr, const double* Rc, long long ldr,
                        double* Sr, double* Sc, long long lds, double* work, hipStream_t s) {
  if (sample_prec == HSS_SAMPLE_F64) {
    launch_sample(A, dtype, n, lda, leaf_of, ncols, Rr, Rc, ldr, Sr, Sc, lds, work, s);
    return hipGetLastError();
  }
  return launch_sample_mixed(static_cast<const float*>(A), n, lda, leaf_of, ncols, sample_prec, Rr, Rc,
                             ldr, Sr, Sc, lds, work, s);
}

hipError_t mark_queued(Handle& H, hipStream_t s) {
  if (!H.queued) {
    const hipError_t e = hipEventCreateWithFlags(&H.queued, hipEventDisableTiming);
    if (e != hipSuccess) {
      H.queued = nullptr;
      return e;
    }
  }
  return hipEventRecord(H.queued, s);
}

// One matvec b = A_HSS x of a batch (Alg. 2).
struct MvJob {
  Handle* H;
  int nrhs;
  const double* x;
  long long ldx;
  double* b;
  long long ldb;
};

// Alg. 2 for several handles at once: every phase (upward sweep of a height,
// downward sweep of a height, leaves) is one batched GEMM launch over all of
// them, heights aligned from the leaves.  Workspace and descriptor staging
// come from the lead handle L.  Host-synchronous at the end (the descriptor
// tables live in the staging area until their copies ran).
hss_status matvec_many(Handle& L, std::vector<MvJob>& jobs, hipStream_t s) {
  L.staging.stream = s;
  // workspace: y (kc), z (kr), w (mr) per node and job, nrhs columns each
  std::vector<std::vector<long long>> oy(jobs.size()), oz(jobs.size()), ow(jobs.size());
  long long tot = 0;
  int maxh = 0;
  for (size_t j = 0; j < jobs.size(); ++j) {
    const std::vector<Node>& nd = jobs[j].H->nodes;
    const int nrhs = jobs[j].nrhs;
    oy[j].resize(nd.size());
    oz[j].resize(nd.size());
    ow[j].resize(nd.size());
    for (size_t t = 0; t < nd.size(); ++t) {
      oy[j][t] = tot;
      tot += (long long)nd[t].kc * nrhs;
      oz[j][t] = tot;
      tot += (long long)nd[t].kr * nrhs;
      ow[j][t] = tot;
      tot += (long long)nd[t].mr * nrhs;
    }
    if (!nd[0].leaf()) maxh = std::max(maxh, jobs[j].H->height);
  }
  double* ws = static_cast<double*>(L.work_mv.ensure((size_t)tot * 8 + 8, s));
  if (!ws) return fail(HSS_ERR_ALLOC, "matvec workspace");
  std::vector<GemmDesc> gd;
  auto flush = [&]() -> hipError_t {
    hipError_t e = gd.empty() ? hipSuccess : launch_gemm_batched(gd.data(), (int)gd.size(), L.staging, s);
    gd.clear();
    return e;
  };
  // upward: y_tau = V^T x_in
  for (int h = 0; h < maxh; ++h) {
    for (size_t j = 0; j < jobs.size(); ++j) {
      const MvJob& J = jobs[j];
      const Handle& H = *J.H;
      const std::vector<Node>& nd = H.nodes;
      if (nd[0].leaf() || h >= H.height) continue;
      const int nrhs = J.nrhs;
      for (int t : H.levels[h]) {
        const Node& v = nd[t];
        Seg src{};
        if (v.leaf()) {
          src = Seg{J.x + (long long)v.lo * J.ldx, nullptr, J.ldx, INT_MAX, nullptr};
        } else {
          src = Seg{ws + oy[j][v.left], ws + oy[j][v.right], nrhs, nd[v.left].kc, nullptr};
        }
        GemmDesc g{};
        g.M = v.kc;
        g.N = nrhs;
        g.K = v.mc - v.kc;
        g.A = v.Ec;
        g.lda = v.kc;
        g.transA = 1;
        g.B = src;
        g.B.map = v.perm_c + v.kc;
        g.C = src;
        g.C.map = v.perm_c;
        g.D = SegOut{ws + oy[j][t], nullptr, nrhs, INT_MAX, nullptr};
        g.alpha = g.beta = 1.0;
        gd.push_back(g);
      }
    }
    HIPCHK(flush());
  }
  // downward: w_tau = U_tau z_tau, then z_a = B_ab y_b + w_tau(top),
  // z_b = B_ba y_a + w_tau(bottom); a handle's root is at its own height
  for (int h = maxh; h >= 1; --h) {
    auto inner_of = [&](const Handle& H) {
      std::vector<int> inner;
      if (h == H.height) inner.push_back(0);
      else if (h < H.height)
        for (int t : H.levels[h]) inner.push_back(t);
      return inner;
    };
    for (size_t j = 0; j < jobs.size(); ++j) {
      const Handle& H = *jobs[j].H;
      if (H.nodes[0].leaf()) continue;
      const int nrhs = jobs[j].nrhs;
      for (int t : inner_of(H)) {
        if (t == 0) continue;
        const Node& v = H.nodes[t];
        GemmDesc g{};  // rows J: w[J[a]] = z[a]
        g.M = v.kr;
        g.N = nrhs;
        g.K = 0;
        g.C = Seg{ws + oz[j][t], nullptr, nrhs, INT_MAX, nullptr};
        g.D = SegOut{ws + ow[j][t], nullptr, nrhs, INT_MAX, v.perm_r};
        g.alpha = 1.0;
        g.beta = 1.0;
        gd.push_back(g);
        GemmDesc e{};  // other rows: w[rest[i]] = (E z)[i]
        e.M = v.mr - v.kr;
        e.N = nrhs;
        e.K = v.kr;
        e.A = v.Er;
        e.lda = v.kr;
        e.B = Seg{ws + oz[j][t], nullptr, nrhs, INT_MAX, nullptr};
        e.D = SegOut{ws + ow[j][t], nullptr, nrhs, INT_MAX, v.perm_r + v.kr};
        e.alpha = 1.0;
        gd.push_back(e);
      }
    }
    HIPCHK(flush());
    for (size_t j = 0; j < jobs.size(); ++j) {
      const Handle& H = *jobs[j].H;
      if (H.nodes[0].leaf()) continue;
      const int nrhs = jobs[j].nrhs;
      for (int t : inner_of(H)) {
        const Node& v = H.nodes[t];
        const Node& a = H.nodes[v.left];
        const Node& c = H.nodes[v.right];
        GemmDesc g{};
        g.N = nrhs;
        g.alpha = 1.0;
        g.beta = (t == 0) ? 0.0 : 1.0;
        // z_a = B_ab y_b (+ w top)
        g.M = a.kr;
        g.K = c.kc;
        g.A = v.B12;
        g.lda = c.kc;
        g.B = Seg{ws + oy[j][v.right], nullptr, nrhs, INT_MAX, nullptr};
        g.C = Seg{ws + ow[j][t], nullptr, nrhs, INT_MAX, nullptr};
        g.D = SegOut{ws + oz[j][v.left], nullptr, nrhs, INT_MAX, nullptr};
        gd.push_back(g);
        // z_b = B_ba y_a (+ w bottom)
        g.M = c.kr;
        g.K = a.kc;
        g.A = v.B21;
        g.lda = a.kc;
        g.B = Seg{ws + oy[j][v.left], nullptr, nrhs, INT_MAX, nullptr};
        g.C = Seg{ws + ow[j][t] + (long long)a.kr * nrhs, nullptr, nrhs, INT_MAX, nullptr};
        g.D = SegOut{ws + oz[j][v.right], nullptr, nrhs, INT_MAX, nullptr};
        gd.push_back(g);
      }
    }
    HIPCHK(flush());
  }
  // leaves: w = U z, then b(I) = w + D x(I); a single-leaf matrix is b = D x
  for (size_t j = 0; j < jobs.size(); ++j) {
    const Handle& H = *jobs[j].H;
    if (H.nodes[0].leaf()) continue;
    const int nrhs = jobs[j].nrhs;
    for (int t : H.leaves) {
      const Node& v = H.nodes[t];
      GemmDesc g{};
      g.M = v.kr;
      g.N = nrhs;
      g.K = 0;
      g.C = Seg{ws + oz[j][t], nullptr, nrhs, INT_MAX, nullptr};
      g.D = SegOut{ws + ow[j][t], nullptr, nrhs, INT_MAX, v.perm_r};
      g.alpha = g.beta = 1.0;
      gd.push_back(g);
      GemmDesc e{};
      e.M = v.mr - v.kr;
      e.N = nrhs;
      e.K = v.kr;
      e.A = v.Er;
      e.lda = v.kr;
      e.B = Seg{ws + oz[j][t], nullptr, nrhs, INT_MAX, nullptr};
      e.D = SegOut{ws + ow[j][t], nullptr, nrhs, INT_MAX, v.perm_r + v.kr};
      e.alpha = 1.0;
      gd.push_back(e);
    }
  }
  HIPCHK(flush());
  for (size_t j = 0; j < jobs.size(); ++j) {
    const MvJob& J = jobs[j];
    const Handle& H = *J.H;
    const std::vector<Node>& nd = H.nodes;
    if (nd[0].leaf()) {
      GemmDesc g{};
      g.M = g.K = (int)H.n;
      g.N = J.nrhs;
      g.A = nd[0].D;
      g.lda = H.n;
      g.B = Seg{J.x, nullptr, J.ldx, INT_MAX, nullptr};
      g.D = SegOut{J.b, nullptr, J.ldb, INT_MAX, nullptr};
      g.alpha = 1.0;
      gd.push_back(g);
      continue;
    }
    for (int t : H.leaves) {
      const Node& v = nd[t];
      GemmDesc g{};
      g.M = g.K = v.size();
      g.N = J.nrhs;
      g.A = v.D;
      g.lda = v.size();
      g.B = Seg{J.x + (long long)v.lo * J.ldx, nullptr, J.ldx, INT_MAX, nullptr};
      g.C = Seg{ws + ow[j][t], nullptr, J.nrhs, INT_MAX, nullptr};
      g.D = SegOut{J.b + (long long)v.lo * J.ldb, nullptr, J.ldb, INT_MAX, nullptr};
      g.alpha = g.beta = 1.0;
      gd.push_back(g);
    }
  }
  HIPCHK(flush());
  // stream-ordered: the descriptor tables stay in their staging block until
  // the work queued so far has run
  HIPCHK(L.staging.retire());
  for (MvJob& J : jobs) HIPCHK(mark_queued(*J.H, s));
  return HSS_OK;
}

hss_status matvec_impl(Handle& H, int nrhs, const double* x, long long ldx, double* b,
                       long long ldb, hipStream_t s) {
  std::vector<MvJob> jobs{MvJob{&H, nrhs, x, ldx, b, ldb}};
  return matvec_many(H, jobs, s);
}

}  // namespace hss

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* hss_last_error(void) { return g_err.c_str(); }

void hss_default_opts(hss_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->rtol = 1e-6;
  o->d0 = 64;
  o->dd = 32;
  o->d_max = 4096;
  o->p_margin = 10;
  o->seed = 0;
  o->leaf_size = 64;
  o->sample_prec = HSS_SAMPLE_F64;
}

hss_status hss_compress(const void* A, int dtype, long long n, long long lda,
                        const hss_tree* tree, const hss_opts* opts, void* stream,
                        hss_handle* out) {
  g_err.clear();
  if (!out) return fail(HSS_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!A || n < 1 || lda < n) return fail(HSS_ERR_ARG, "A, n or lda invalid");
  if (dtype != HSS_F64 && dtype != HSS_F32) return fail(HSS_ERR_ARG, "dtype");
  if (n > INT_MAX / 2) return fail(HSS_ERR_ARG, "n too large");
  hss_opts o;
  if (opts) o = *opts;
  else hss_default_opts(&o);
  if (!(o.rtol >= 0.0) || o.d0 < 1 || o.dd < 1 || o.d_max < o.d0 || o.p_margin < 0)
    return fail(HSS_ERR_ARG, "rtol / d0 / dd / d_max / p_margin invalid");
  if (o.sample_prec != HSS_SAMPLE_F64 && o.sample_prec != HSS_SAMPLE_F32 &&
      o.sample_prec != HSS_SAMPLE_BF16X3)
    return fail(HSS_ERR_ARG, "unknown sample precision");
  if (o.sample_prec != HSS_SAMPLE_F64 && dtype != HSS_F32)
    return fail(HSS_ERR_ARG, "reduced-precision sampling needs A stored in FP32");
  if ((o.R_user_r == nullptr) != (o.R_user_c == nullptr))
    return fail(HSS_ERR_ARG, "R_user_r and R_user_c must both be given or both NULL");
  if (o.R_user_r && o.ld_R_user < o.d_max) return fail(HSS_ERR_ARG, "ld_R_user < d_max");
  hss_handle_s* p = nullptr;
  CHK(new_handle(out, n, static_cast<hipStream_t>(stream), &p));
  Handle& H = p->h;
  H.dtype = dtype;
  H.opts = o;
  {
    const char* v = std::getenv("HSS_VERBOSE");
    H.verbose = verbose_level(v);
  }
  hss_status st = build_tree(H, n, tree, o.leaf_size);
  if (st == HSS_OK) st = compress_impl(H, A, lda);
  if (st != HSS_OK && st != HSS_NOT_CONVERGED) {
    const std::string msg = g_err;
    free_handle(p);
    g_err = msg;
    return st;
  }
  *out = p;
  return st;
}

hss_status hss_compress_batched(int nmat, const void* const* A, int dtype, const long long* n,
                                const long long* lda, const hss_tree* trees, const hss_opts* opts,
                                void* stream, hss_handle* out, int* status) {
  return hss::compress_batched(nmat, A, dtype, n, lda, trees, opts, stream, out, status, true);
}

}  // extern "C"

hss_status hss::compress_batched(int nmat, const void* const* A, int dtype, const long long* n,
                                 const long long* lda, const hss_tree* trees, const hss_opts* opts,
                                 void* stream, hss_handle* out, int* status, bool share_arena) {
  g_err.clear();
  if (nmat < 1 || !A || !n || !lda || !out) return fail(HSS_ERR_ARG, "batch arguments");
  if (dtype != HSS_F64 && dtype != HSS_F32) return fail(HSS_ERR_ARG, "dtype");
  hss_opts o;
  if (opts) o = *opts;
  else hss_default_opts(&o);
  if (!(o.rtol >= 0.0) || o.d0 < 1 || o.dd < 1 || o.d_max < o.d0 || o.p_margin < 0)
    return fail(HSS_ERR_ARG, "rtol / d0 / dd / d_max / p_margin invalid");
  if (o.sample_prec < HSS_SAMPLE_F64 || o.sample_prec > HSS_SAMPLE_BF16X3)
    return fail(HSS_ERR_ARG, "unknown sample precision");
  if (o.sample_prec != HSS_SAMPLE_F64 && dtype != HSS_F32)
    return fail(HSS_ERR_ARG, "reduced-precision sampling needs A stored in FP32");
  if (o.R_user_r || o.R_user_c) return fail(HSS_ERR_ARG, "no user random matrices in a batch");
  for (int i = 0; i < nmat; ++i) {
    out[i] = nullptr;
    if (!A[i] || n[i] < 1 || lda[i] < n[i] || n[i] > INT_MAX / 2)
      return fail(HSS_ERR_ARG, "matrix " + std::to_string(i) + ": A, n or lda invalid");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<hss_handle_s*> hs(nmat, nullptr);
  auto free_all = [&]() {
    const std::string msg = g_err;
    for (hss_handle_s* p : hs) free_handle(p);
    g_err = msg;
  };
  const char* v = std::getenv("HSS_VERBOSE");
  std::vector<Job> jobs(nmat);
  for (int i = 0; i < nmat; ++i) {
    hss_status st = new_handle(&out[i], n[i], s, &hs[i]);
    if (st == HSS_OK) {
      Handle& H = hs[i]->h;
      H.dtype = dtype;
      H.opts = o;
      H.verbose = verbose_level(v);
      if (share_arena) {  // one generator arena for the batch
        if (i == 0) H.gen->chunk = (size_t)64 << 20;
        else H.gen = hs[0]->h.gen;
      }
      st = build_tree(H, n[i], trees ? &trees[i] : nullptr, o.leaf_size);
      jobs[i].H = &H;
      jobs[i].A = A[i];
      jobs[i].lda = lda[i];
    }
    if (st != HSS_OK) {
      free_all();
      return st;
    }
  }
  const hss_status st = compress_batch(jobs);
  if (st != HSS_OK) {
    free_all();
    return st;
  }
  bool all = true;
  for (int i = 0; i < nmat; ++i) {
    out[i] = hs[i];
    const bool c = hs[i]->h.converged;
    all = all && c;
    if (status) status[i] = c ? HSS_OK : HSS_NOT_CONVERGED;
  }
  return all ? HSS_OK : HSS_NOT_CONVERGED;
}

extern "C" {

hss_status hss_matvec(hss_handle h, int nrhs, const double* x, long long ldx, double* b,
                      long long ldb, void* stream) {
  g_err.clear();
  if (!h || !h->h.compressed) return fail(HSS_ERR_STATE, "handle not compressed");
  if (nrhs < 0 || ldx < nrhs || ldb < nrhs) return fail(HSS_ERR_ARG, "nrhs / ldx / ldb");
  if (nrhs == 0) return HSS_OK;
  if (!x || !b) return fail(HSS_ERR_ARG, "x or b is NULL");
  const Handle& H = h->h;
  const char* xb = reinterpret_cast<const char*>(x);
  const char* bb = reinterpret_cast<const char*>(b);
  const long long xe = ((H.n - 1) * ldx + nrhs) * 8, be = ((H.n - 1) * ldb + nrhs) * 8;
  if (xb < bb + be && bb < xb + xe) return fail(HSS_ERR_ARG, "x and b overlap");
  return matvec_impl(h->h, nrhs, x, ldx, b, ldb, static_cast<hipStream_t>(stream));
}

hss_status hss_matvec_batched(int nmat, const hss_handle* h, int nrhs, const double* const* x,
                              const long long* ldx, double* const* b, const long long* ldb,
                              void* stream) {
  g_err.clear();
  if (nmat < 0 || (nmat > 0 && (!h || !x || !ldx || !b || !ldb)))
    return fail(HSS_ERR_ARG, "batch arguments");
  if (nrhs < 0) return fail(HSS_ERR_ARG, "nrhs");
  if (nmat == 0 || nrhs == 0) return HSS_OK;
  std::vector<MvJob> jobs;
  jobs.reserve(nmat);
  for (int i = 0; i < nmat; ++i) {
    const std::string tag = "matrix " + std::to_string(i) + ": ";
    if (!h[i] || !h[i]->h.compressed) return fail(HSS_ERR_STATE, tag + "handle not compressed");
    if (ldx[i] < nrhs || ldb[i] < nrhs) return fail(HSS_ERR_ARG, tag + "ldx / ldb");
    if (!x[i] || !b[i]) return fail(HSS_ERR_ARG, tag + "x or b is NULL");
    const long long n = h[i]->h.n;
    const char* xb = reinterpret_cast<const char*>(x[i]);
    const char* bb = reinterpret_cast<const char*>(b[i]);
    const long long xe = ((n - 1) * ldx[i] + nrhs) * 8, be = ((n - 1) * ldb[i] + nrhs) * 8;
    if (xb < bb + be && bb < xb + xe) return fail(HSS_ERR_ARG, tag + "x and b overlap");
    for (int q = 0; q < i; ++q)
      if (h[q] == h[i]) return fail(HSS_ERR_ARG, tag + "handle appears twice");
    jobs.push_back(MvJob{&h[i]->h, nrhs, x[i], ldx[i], b[i], ldb[i]});
  }
  return matvec_many(h[0]->h, jobs, static_cast<hipStream_t>(stream));
}

hss_status hss_stats(hss_handle h, hss_stats_t* st) {
  if (!h || !st) return fail(HSS_ERR_ARG, "NULL argument");
  const Handle& H = h->h;
  std::memset(st, 0, sizeof(*st));
  st->n = H.n;
  st->n_nodes = (int)H.nodes.size();
  st->height = H.height;
  st->d_final = H.d;
  st->passes = H.passes;
  st->converged = H.converged ? 1 : 0;
  int mx = 0;
  for (size_t t = 1; t < H.nodes.size(); ++t) mx = std::max(mx, std::max(H.nodes[t].kr, H.nodes[t].kc));
  st->max_rank = mx;
  st->generator_bytes = H.generator_bytes();
  st->sample_flops = 4.0 * (double)H.n * (double)H.n * (double)H.d;
  st->t_total_ms = H.t_total;
  st->t_sample_ms = H.t_sample;
  st->t_levels_ms = H.t_levels;
  st->t_id_ms = H.t_id;
  st->n_sample_launches = H.n_sgemm;
  st->t_sample_gemm_ms = H.t_sgemm;
  st->sample_gemm_flops = H.sgemm_flops;
  st->sample_gemm_bytes = H.sgemm_bytes;
  st->id_flops = H.id_flops;
  st->t_level_gemm_ms = H.t_lgemm;
  st->level_gemm_bytes = H.lgemm_bytes;
  st->t_gather_ms = H.t_gather;
  st->gather_bytes = H.gather_bytes;
  return HSS_OK;
}

hss_status hss_ranks(hss_handle h, int* kr, int* kc, int* mr, int* mc) {
  if (!h) return fail(HSS_ERR_ARG, "NULL handle");
  const Handle& H = h->h;
  for (size_t t = 0; t < H.nodes.size(); ++t) {
    const Node& v = H.nodes[t];
    if (kr) kr[t] = t ? v.kr : 0;
    if (kc) kc[t] = t ? v.kc : 0;
    if (mr) mr[t] = v.leaf() ? v.size() : v.mr;
    if (mc) mc[t] = v.leaf() ? v.size() : v.mc;
  }
  return HSS_OK;
}

hss_status hss_export_node(hss_handle h, int node, hss_node_generators* g) {
  if (!h || !g) return fail(HSS_ERR_ARG, "NULL argument");
  Handle& H = h->h;
  if (node < 0 || node >= (int)H.nodes.size()) return fail(HSS_ERR_ARG, "node out of range");
  const Node& v = H.nodes[node];
  HIPCHK(hipStreamSynchronize(H.stream));
  if (node != 0) {
    if (g->Jr && v.kr) HIPCHK(hipMemcpy(g->Jr, v.perm_r, (size_t)v.kr * 4, hipMemcpyDeviceToHost));
    if (g->Jc && v.kc) HIPCHK(hipMemcpy(g->Jc, v.perm_c, (size_t)v.kc * 4, hipMemcpyDeviceToHost));
    if (g->Er && v.kr && v.mr > v.kr)
      HIPCHK(hipMemcpy(g->Er, v.Er, (size_t)(v.mr - v.kr) * v.kr * 8, hipMemcpyDeviceToHost));
    if (g->Ec && v.kc && v.mc > v.kc)
      HIPCHK(hipMemcpy(g->Ec, v.Ec, (size_t)(v.mc - v.kc) * v.kc * 8, hipMemcpyDeviceToHost));
    if (g->Ir && v.kr && v.Ir) HIPCHK(hipMemcpy(g->Ir, v.Ir, (size_t)v.kr * 4, hipMemcpyDeviceToHost));
    if (g->Ic && v.kc && v.Ic) HIPCHK(hipMemcpy(g->Ic, v.Ic, (size_t)v.kc * 4, hipMemcpyDeviceToHost));
  }
  if (v.leaf() && g->D)
    HIPCHK(hipMemcpy(g->D, v.D, (size_t)v.size() * v.size() * 8, hipMemcpyDeviceToHost));
  if (!v.leaf()) {
    const Node& a = H.nodes[v.left];
    const Node& c = H.nodes[v.right];
    if (g->B12 && a.kr && c.kc)
      HIPCHK(hipMemcpy(g->B12, v.B12, (size_t)a.kr * c.kc * 8, hipMemcpyDeviceToHost));
    if (g->B21 && c.kr && a.kc)
      HIPCHK(hipMemcpy(g->B21, v.B21, (size_t)c.kr * a.kc * 8, hipMemcpyDeviceToHost));
  }
  return HSS_OK;
}

hss_status hss_import(long long n, const hss_tree* tree, const int* kr, const int* kc,
                      const hss_node_generators* nodes, hss_handle* out) {
  g_err.clear();
  if (!out || !tree || !kr || !kc || !nodes || n < 1) return fail(HSS_ERR_ARG, "NULL argument");
  *out = nullptr;
  hss_handle_s* p = nullptr;
  CHK(new_handle(out, n, nullptr, &p));
  Handle& H = p->h;
  hss_status st = build_tree(H, n, tree, 1);
  if (st != HSS_OK) {
    free_handle(p);
    return st;
  }
  std::vector<Node>& nd = H.nodes;
  auto bad = [&](const char* m) {
    free_handle(p);
    return fail(HSS_ERR_ARG, m);
  };
  // sizes bottom-up
  std::vector<int> order;
  for (int h = 0; h < H.height; ++h)
    for (int t : H.levels[h]) order.push_back(t);
  order.push_back(0);
  for (int t : order) {
    Node& v = nd[t];
    if (v.leaf()) v.mr = v.mc = v.size();
    else {
      v.mr = nd[v.left].kr + nd[v.right].kr;
      v.mc = nd[v.left].kc + nd[v.right].kc;
    }
    if (t != 0) {
      v.kr = kr[t];
      v.kc = kc[t];
      if (v.kr < 0 || v.kc < 0 || v.kr > v.mr || v.kc > v.mc) return bad("rank out of range");
    }
  }
  for (int t : order) {
    Node& v = nd[t];
    const hss_node_generators& g = nodes[t];
    if (v.leaf()) {
      v.D = arena_alloc<double>(H, (size_t)v.size() * v.size());
      if (!v.D || !g.D) return bad("leaf D missing");
      if (hipMemcpy(v.D, g.D, (size_t)v.size() * v.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return bad("copy D");
    } else {
      const Node& a = nd[v.left];
      const Node& c = nd[v.right];
      v.B12 = arena_alloc<double>(H, (size_t)a.kr * c.kc);
      v.B21 = arena_alloc<double>(H, (size_t)c.kr * a.kc);
      if ((a.kr * c.kc && !g.B12) || (c.kr * a.kc && !g.B21)) return bad("B missing");
      if (a.kr * c.kc &&
          hipMemcpy(v.B12, g.B12, (size_t)a.kr * c.kc * 8, hipMemcpyHostToDevice) != hipSuccess)
        return bad("copy B12");
      if (c.kr * a.kc &&
          hipMemcpy(v.B21, g.B21, (size_t)c.kr * a.kc * 8, hipMemcpyHostToDevice) != hipSuccess)
        return bad("copy B21");
    }
    if (t == 0) continue;
    for (int side = 0; side < 2; ++side) {
      const int m = side ? v.mc : v.mr, k = side ? v.kc : v.kr;
      const int* J = side ? g.Jc : g.Jr;
      const double* E = side ? g.Ec : g.Er;
      if (k && !J) return bad("J missing");
      if (k && m > k && !E) return bad("E missing");
      std::vector<int> perm;
      std::vector<char> sel(m, 0);
      for (int q = 0; q < k; ++q) {
        if (J[q] < 0 || J[q] >= m || sel[J[q]]) return bad("J is not a set of distinct rows");
        sel[J[q]] = 1;
        perm.push_back(J[q]);
      }
      for (int q = 0; q < m; ++q)
        if (!sel[q]) perm.push_back(q);
      int* dp = arena_alloc<int>(H, (size_t)m);
      double* de = arena_alloc<double>(H, (size_t)(m - k) * k + 1);
      if (!dp || !de) return bad("alloc");
      if (m && hipMemcpy(dp, perm.data(), (size_t)m * 4, hipMemcpyHostToDevice) != hipSuccess)
        return bad("copy permutation");
      if ((m - k) * k && hipMemcpy(de, E, (size_t)(m - k) * k * 8, hipMemcpyHostToDevice) != hipSuccess)
        return bad("copy E");
      if (side) {
        v.perm_c = dp;
        v.Ec = de;
      } else {
        v.perm_r = dp;
        v.Er = de;
      }
    }
    v.state = HSS_COMPRESSED;
  }
  H.compressed = true;
  H.d = 0;
  *out = p;
  return HSS_OK;
}

void hss_destroy(hss_handle h) { free_handle(h); }

hss_status hss_set_allocator(hss_alloc_fn alloc, hss_free_fn free_fn, void* ctx) {
  g_err.clear();
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(HSS_ERR_ARG, "alloc and free must both be given or both be NULL");
  std::lock_guard<std::mutex> lk(g_user_mu);
  g_user.alloc = alloc;
  g_user.free = free_fn;
  g_user.ctx = alloc ? ctx : nullptr;
  return HSS_OK;
}

hss_status hss_release_cached_memory(void) {
  g_err.clear();
  HIPCHK(hss::release_cached_memory());
  return HSS_OK;
}

hss_status hss_random_normal(unsigned long long seed, int which, long long n, int col0, int col1,
                             int sample_prec, double* R, long long ld, void* stream) {
  g_err.clear();
  if (n < 0 || col0 < 0 || col1 < col0 || (n > 0 && !R) || ld < col1 - col0 || (which != 0 && which != 1))
    return fail(HSS_ERR_ARG, "random_normal arguments");
  if (sample_prec < HSS_SAMPLE_F64 || sample_prec > HSS_SAMPLE_BF16X3)
    return fail(HSS_ERR_ARG, "unknown sample precision");
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_random_normal(seed, which, n, col0, col1, R, ld, s);
  launch_round_r(R, ld, n, 0, col1 - col0, sample_prec, s);
  HIPCHK(hipGetLastError());
  return HSS_OK;
}

hss_status hss_sample(const void* A, int dtype, int sample_prec, long long n, long long lda,
                      const int* leaf_of, int ncols, const double* Rr, const double* Rc,
                      long long ldr, double* Sr, double* Sc, long long lds, void* stream) {
  g_err.clear();
  long long wd = 0;
  CHK(sample_args(A, dtype, sample_prec, n, lda, ncols, Rr, Rc, ldr, Sr, Sc, lds, &wd));
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* work = nullptr;
  if (wd > 0) {
    work = static_cast<double*>(pool_alloc((size_t)wd * 8, s));
    if (!work) return fail(HSS_ERR_ALLOC, "sampling workspace");
  }
  const hipError_t e = sample_queue(A, dtype, sample_prec, n, lda, leaf_of, ncols, Rr, Rc, ldr, Sr, Sc,
                                    lds, work, s);
  pool_free(work, s);  // stream-ordered: reused only after the products ran
  HIPCHK(e);
  return HSS_OK;
}

hss_status hss_gemm_batched(int nprob, const int* M, const int* N, const int* K, const double* const* A,
                            const long long* lda, const int* transA, const double* const* B,
                            const long long* ldb, double* const* C, const long long* ldc, double alpha,
                            double beta, int variant, void* stream) {
  g_err.clear();
  if (nprob < 0 || (nprob > 0 && (!M || !N || !K || !A || !lda || !transA || !B || !ldb || !C || !ldc)))
    return fail(HSS_ERR_ARG, "gemm arguments");
  if (variant >= gemm_variants()) return fail(HSS_ERR_ARG, "gemm variant out of range");
  std::vector<GemmDesc> gd(nprob);
  for (int p = 0; p < nprob; ++p) {
    if (M[p] < 0 || N[p] < 0 || K[p] < 0 || ldb[p] < N[p] || ldc[p] < N[p] ||
        lda[p] < (transA[p] ? M[p] : K[p]))
      return fail(HSS_ERR_ARG, "gemm problem " + std::to_string(p) + ": sizes");
    if ((M[p] > 0 && N[p] > 0) && (!C[p] || (K[p] > 0 && (!A[p] || !B[p]))))
      return fail(HSS_ERR_ARG, "gemm problem " + std::to_string(p) + ": NULL pointer");
    GemmDesc& g = gd[p];
    g.M = M[p];
    g.N = N[p];
    g.K = K[p];
    g.A = A[p];
    g.lda = lda[p];
    g.transA = transA[p] ? 1 : 0;
    g.B = Seg{B[p], nullptr, ldb[p], INT_MAX, nullptr};
    g.C = Seg{C[p], nullptr, ldc[p], INT_MAX, nullptr};
    g.D = SegOut{C[p], nullptr, ldc[p], INT_MAX, nullptr};
    g.alpha = alpha;
    g.beta = beta;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // descriptor tables: a process-wide staging area whose blocks are retired
  // behind an event after each call (stream-ordered, no wait)
  static std::mutex mu;
  static Staging st;
  std::lock_guard<std::mutex> lk(mu);
  st.stream = s;
  hipError_t e = launch_gemm_batched(gd.data(), nprob, st, s, variant);
  if (e == hipSuccess) e = st.retire();
  HIPCHK(e);
  return HSS_OK;
}

int hss_gemm_variants(void) { return gemm_variants(); }

hss_status hss_id_batched(int nprob, const double* const* ys, const int* m, const int* d,
                          const long long* ldy, double rtol, int* const* perms,
                          double* const* es, int* k, void* stream) {
  g_err.clear();
  if (nprob < 0 || (nprob > 0 && (!ys || !m || !d || !ldy || !perms || !es || !k)))
    return fail(HSS_ERR_ARG, "id arguments");
  if (nprob == 0) return HSS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<IdProblem> pr(nprob);
  for (int q = 0; q < nprob; ++q) {
    if (m[q] < 0 || d[q] < 0 || (m[q] > 0 && d[q] > 0 && ldy[q] < d[q]))
      return fail(HSS_ERR_ARG, "problem sizes");
    pr[q].Y = ys[q];
    pr[q].ldy = ldy[q];
    pr[q].m = m[q];
    pr[q].d = d[q];
    pr[q].perm = perms[q];
    pr[q].E = es[q];
    pr[q].kfail = -1;
  }
  Staging st;
  HIPCHK(st.init((size_t)1 << 20, s));
  const size_t wb = id_workspace_bytes(pr.data(), nprob);
  void* base = pool_alloc(wb, s);
  if (!base) {
    st.release();
    return fail(HSS_ERR_ALLOC, "id workspace");
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = launch_id_factor(pr.data(), nprob, rtol, base, wb, k, st, s);
  std::vector<int> sel(nprob);
  for (int q = 0; q < nprob; ++q) sel[q] = q;
  if (e == hipSuccess) e = launch_id_finish(pr.data(), nprob, k, sel.data(), nprob, base, st, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  pool_free(base, s);
  st.release();
  HIPCHK(e);
  return HSS_OK;
}

}  // extern "C"

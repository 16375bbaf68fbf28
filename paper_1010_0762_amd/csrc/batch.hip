// Continuous batching of the iteration launches of several solves (batch.h).
//
// Solves attached to one batch run on their own host threads and HIP streams
// as before; only their chunks of iterations change hands.  A solve hands in
// its chunk (the per-iteration kernel arguments it would have launched with)
// and waits; the first waiting thread that finds every iterating solve's
// chunk in hand -- or the oldest chunk older than the batch's window --
// launches all chunks in hand on the batch stream: per iteration one
// k_it1_multi and one k_it2_multi over every chunk that still has that
// iteration, then one k_itfin_multi, each slot's blocks a contiguous range
// starting on a multiple of 8 (the XCD count).  The batch stream waits for
// each solve's stream first; each solve's stream then waits for the batch.
// The per-slot arithmetic is that of the single-solve kernels (same bodies,
// the slot's own block index and count), so a solve gives the same bits
// alone and in a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.h"
#include "errors.h"

#define TRY_B(call)      \
  do {                   \
    const int r_ = call; \
    if (r_ < 0) return r_; \
  } while (0)

#define B_HIPCHECK(call)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return rbicg_fail(RBICG_EHIP, "%s failed at %s:%d: %s", #call, __FILE__, __LINE__, \
                        hipGetErrorString(e_));                                           \
  } while (0)

namespace {

using clk = std::chrono::steady_clock;

struct Pending {
  BatchChunk *c = nullptr;
  hipEvent_t in = nullptr;
  bool done = false;
  int rc = 0;
};

constexpr int NBUF = 8;  // table buffers in flight
constexpr int NSTREAM = 4;  // batch streams (launches rotate over them)
constexpr int NGRAPH = 64;  // captured launch sets kept (least recently used dropped)

// A launch set as a graph: the kernels of one batch launch, replayed whenever
// the same table buffer holds tables of the same shape (the kernels read
// their arguments from the tables, so only the table contents change).
struct Captured {
  hipGraphExec_t exec = nullptr;
  long last = 0;
};

}  // namespace

struct rbicg_batch_s {
  std::mutex mu;
  std::condition_variable cv;
  hipStream_t sts[NSTREAM] = {};
  hipStream_t st = nullptr;  // stream of the launch being built
  int max_slots = RBICG_BATCH_SLOTS;
  std::chrono::microseconds window{50};
  int active = 0;
  std::vector<Pending *> pending;
  clk::time_point first_t;
  bool launching = false;
  std::vector<hipEvent_t> events;  // pool of hand-in events
  // argument tables: pinned staging and device copies, ring of NBUF
  char *host[NBUF] = {};
  char *dev[NBUF] = {};
  size_t cap[NBUF] = {};
  hipEvent_t used[NBUF] = {};
  int next = 0;
  hipEvent_t fin = nullptr;
  // statistics: launches, chunks, slot-iterations, largest batch, graph
  // replays, graph captures
  double stat[6] = {0, 0, 0, 0, 0, 0};
  // launch sets captured as HIP graphs, keyed by table buffer and shape
  bool graphs = false;
  std::map<std::vector<long>, Captured> cap_sets;
  long uses = 0;
};

namespace {

hipEvent_t take_event(rbicg_batch b) {
  std::lock_guard<std::mutex> lk(b->mu);
  if (b->events.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = b->events.back();
  b->events.pop_back();
  return e;
}

constexpr size_t al16(size_t b) { return (b + 15) / 16 * 16; }

// Argument types of a kind.
template <int K> struct KindT;
template <> struct KindT<BK_F64> { using V = double; using M = double; };
template <> struct KindT<BK_C128_REAL_A> { using V = cd; using M = double; };
template <> struct KindT<BK_C128> { using V = cd; using M = cd; };
template <> struct KindT<BK_F32> { using V = float; using M = float; };

// Tables and launches of one group (one kind, one rows-per-thread mode).
// One launch of a launch set: directly on the batch stream, or as a node of
// a graph chained after the previous one.
struct Op {
  std::function<void()> launch;
  std::function<hipError_t(hipGraph_t, hipGraphNode_t &)> node;
};

template <int K>
int launch_group(rbicg_batch b, const std::vector<Pending *> &g, bool one_row, char *hbase,
                 char *dbase, size_t &off, std::vector<Op> &launches, std::vector<long> &shape) {
  using V = typename KindT<K>::V;
  using M = typename KindT<K>::M;
  using A1 = It1Args<V, M>;
  using A2 = It2Args<V>;
  int maxlen = 0;
  size_t lds = 0;
  for (auto *p : g) {
    maxlen = std::max(maxlen, p->c->len);
    lds = std::max(lds, p->c->lds);
  }
  const hipStream_t st = b->st;
  // per iteration: a contiguous array of A1 for the slots that still run it,
  // then one of A2 (each array starts on 16 bytes)
  for (int t = 0; t < maxlen; ++t) {
    off = al16(off);
    const size_t o1 = off;
    int ns = 0, b0 = 0;
    for (auto *p : g) {
      if (t >= p->c->len) continue;
      A1 a;
      std::memcpy(&a, p->c->it1.data() + (size_t)t * sizeof(A1), sizeof(A1));
      a.b0 = b0;
      a.nb = p->c->nb;
      std::memcpy(hbase + off, &a, sizeof(A1));
      off += sizeof(A1);
      b0 += (p->c->nb + 7) / 8 * 8;
      ++ns;
    }
    const int nblk = b0;
    off = al16(off);
    const size_t o2 = off;
    b0 = 0;
    for (auto *p : g) {
      if (t >= p->c->len) continue;
      A2 a;
      std::memcpy(&a, p->c->it2.data() + (size_t)t * sizeof(A2), sizeof(A2));
      a.b0 = b0;
      a.nb = p->c->nb;
      std::memcpy(hbase + off, &a, sizeof(A2));
      off += sizeof(A2);
      b0 += (p->c->nb + 7) / 8 * 8;
    }
    const A1 *d1 = (const A1 *)(dbase + o1);
    const A2 *d2 = (const A2 *)(dbase + o2);
    shape.insert(shape.end(), {K, one_row ? 1L : 0L, (long)o1, (long)o2, ns, nblk, (long)lds});
    launches.push_back({[=]() {
                          launch_it1_multi<V, M>(st, d1, ns, nblk, lds, one_row);
                          launch_it2_multi<V>(st, d2, ns, nblk);
                        },
                        [=](hipGraph_t gr, hipGraphNode_t &last) {
                          hipError_t e = graph_it1_multi<V, M>(gr, last, d1, ns, nblk, lds, one_row);
                          if (e == hipSuccess) e = graph_it2_multi<V>(gr, last, d2, ns, nblk);
                          return e;
                        }});
  }
  off = al16(off);
  const size_t of = off;
  for (auto *p : g) {
    std::memcpy(hbase + off, &p->c->fin, sizeof(ItfinArgs));
    off += sizeof(ItfinArgs);
  }
  const ItfinArgs *df = (const ItfinArgs *)(dbase + of);
  const int n = (int)g.size();
  shape.insert(shape.end(), {-K - 1, (long)of, n});
  launches.push_back({[=]() { launch_itfin_multi<V>(st, df, n); },
                      [=](hipGraph_t gr, hipGraphNode_t &last) { return graph_itfin_multi<V>(gr, last, df, n); }});
  return 0;
}

// Run the launches: directly, or as a HIP graph captured once per table
// buffer and shape and replayed afterwards (kernels only; no memory nodes).
int run_launches(rbicg_batch b, std::vector<Op> &launches, std::vector<long> key) {
  if (!b->graphs) {
    for (auto &f : launches) f.launch();
    B_HIPCHECK(hipGetLastError());
    return 0;
  }
  ++b->uses;
  auto it = b->cap_sets.find(key);
  if (it == b->cap_sets.end()) {
    if ((int)b->cap_sets.size() >= NGRAPH) {  // drop the least recently used
      auto lru = b->cap_sets.begin();
      for (auto jt = b->cap_sets.begin(); jt != b->cap_sets.end(); ++jt)
        if (jt->second.last < lru->second.last) lru = jt;
      (void)hipGraphExecDestroy(lru->second.exec);
      b->cap_sets.erase(lru);
    }
    // built node by node (no stream capture: other threads keep using
    // their streams, the null stream included, while a graph is built)
    hipGraph_t g = nullptr;
    B_HIPCHECK(hipGraphCreate(&g, 0));
    hipGraphNode_t last = nullptr;
    for (auto &f : launches) {
      const hipError_t e = f.node(g, last);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return rbicg_fail(RBICG_EHIP, "batch graph node: %s", hipGetErrorString(e));
      }
    }
    Captured c;
    const hipError_t ie = hipGraphInstantiate(&c.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return rbicg_fail(RBICG_EHIP, "batch graph instantiation failed: %s", hipGetErrorString(ie));
    it = b->cap_sets.emplace(std::move(key), c).first;
    b->stat[5] += 1;
  } else {
    b->stat[4] += 1;
  }
  it->second.last = b->uses;
  B_HIPCHECK(hipGraphLaunch(it->second.exec, b->st));
  return 0;
}

size_t group_bytes(const std::vector<Pending *> &g, size_t a1, size_t a2) {
  size_t tot = 0, maxlen = 0;
  for (auto *p : g) {
    tot += (size_t)p->c->len * (a1 + a2) + sizeof(ItfinArgs);
    maxlen = std::max(maxlen, (size_t)p->c->len);
  }
  return tot + 32 * (maxlen + 1) + 64;  // alignment of each array
}

// Enqueue the chunks in take on the batch stream (called by one thread at a
// time, without the batch lock).
int launch(rbicg_batch b, std::vector<Pending *> &take) {
  // launches rotate over the batch streams, so that a long launch does not
  // hold up the next one (each slot's chunks stay ordered through its own
  // stream's events)
  b->st = b->sts[(int)b->stat[0] % NSTREAM];
  // the batch runs after every slot's prior work
  for (auto *p : take) B_HIPCHECK(hipStreamWaitEvent(b->st, p->in, 0));
  // groups by kind and rows-per-thread mode, in hand-in order
  std::vector<std::vector<Pending *>> groups(2 * BK_KINDS);
  for (auto *p : take) groups[2 * p->c->kind + (p->c->one_row ? 1 : 0)].push_back(p);
  size_t need = 0;
  for (int gi = 0; gi < 2 * BK_KINDS; ++gi) {
    if (groups[gi].empty()) continue;
    const int kind = gi / 2;
    const size_t a1 = kind == BK_F64 ? sizeof(It1Args<double, double>)
                      : kind == BK_C128_REAL_A ? sizeof(It1Args<cd, double>)
                      : kind == BK_C128 ? sizeof(It1Args<cd, cd>)
                                        : sizeof(It1Args<float, float>);
    const size_t a2 = kind == BK_F32 ? sizeof(It2Args<float>)
                      : kind == BK_F64 ? sizeof(It2Args<double>) : sizeof(It2Args<cd>);
    need += group_bytes(groups[gi], a1, a2);
  }
  // a table buffer whose previous batch has finished
  const int bi = b->next;
  b->next = (b->next + 1) % NBUF;
  if (b->used[bi]) B_HIPCHECK(hipEventSynchronize(b->used[bi]));
  if (b->cap[bi] < need) {
    if (b->host[bi]) (void)hipHostFree(b->host[bi]);
    if (b->dev[bi]) (void)hipFree(b->dev[bi]);
    b->host[bi] = nullptr;
    b->dev[bi] = nullptr;
    b->cap[bi] = 0;
    const size_t c = std::max<size_t>(need * 2, 1 << 16);
    B_HIPCHECK(hipHostMalloc((void **)&b->host[bi], c, hipHostMallocDefault));
    B_HIPCHECK(hipMalloc((void **)&b->dev[bi], c));
    b->cap[bi] = c;
  }
  std::vector<Op> launches;
  std::vector<long> shape{bi};  // the table buffer, then the launches' shape
  size_t off = 0;
  for (int gi = 0; gi < 2 * BK_KINDS; ++gi) {
    const auto &g = groups[gi];
    if (g.empty()) continue;
    const bool one_row = gi % 2 == 1;
    int rc = 0;
    switch (gi / 2) {
      case BK_F64: rc = launch_group<BK_F64>(b, g, one_row, b->host[bi], b->dev[bi], off, launches, shape); break;
      case BK_C128_REAL_A:
        rc = launch_group<BK_C128_REAL_A>(b, g, one_row, b->host[bi], b->dev[bi], off, launches, shape);
        break;
      case BK_C128: rc = launch_group<BK_C128>(b, g, one_row, b->host[bi], b->dev[bi], off, launches, shape); break;
      default: rc = launch_group<BK_F32>(b, g, one_row, b->host[bi], b->dev[bi], off, launches, shape); break;
    }
    if (rc < 0) return rc;
  }
  if (off > b->cap[bi]) return rbicg_fail(RBICG_EINVAL, "batch tables overflow their buffer");
  B_HIPCHECK(hipMemcpyAsync(b->dev[bi], b->host[bi], off, hipMemcpyHostToDevice, b->st));
  // a reallocated buffer changes the tables' addresses: its graphs are stale
  shape.push_back((long)(uintptr_t)b->dev[bi]);
  TRY_B(run_launches(b, launches, std::move(shape)));
  if (!b->used[bi]) B_HIPCHECK(hipEventCreateWithFlags(&b->used[bi], hipEventDisableTiming));
  B_HIPCHECK(hipEventRecord(b->used[bi], b->st));
  // every slot's stream continues after the batch
  for (auto *p : take) B_HIPCHECK(hipStreamWaitEvent(p->c->st, b->used[bi], 0));
  return 0;
}

}  // namespace

void batch_enter(rbicg_batch b) {
  std::lock_guard<std::mutex> lk(b->mu);
  ++b->active;
}

void batch_leave(rbicg_batch b) {
  std::lock_guard<std::mutex> lk(b->mu);
  --b->active;
  b->cv.notify_all();
}

int batch_submit(rbicg_batch b, BatchChunk &c) {
  Pending p;
  p.c = &c;
  p.in = take_event(b);
  if (!p.in) return rbicg_fail(RBICG_EHIP, "hipEventCreate failed");
  B_HIPCHECK(hipEventRecord(p.in, c.st));
  std::unique_lock<std::mutex> lk(b->mu);
  if (b->pending.empty()) b->first_t = clk::now();
  b->pending.push_back(&p);
  b->cv.notify_all();
  while (!p.done) {
    const int np = (int)b->pending.size();
    const bool all_in = np >= std::max(1, b->active) || np >= b->max_slots;
    const bool late = clk::now() >= b->first_t + b->window;
    if (!b->launching && np > 0 && (all_in || late)) {
      b->launching = true;
      const int nt = std::min(np, b->max_slots);
      std::vector<Pending *> take(b->pending.begin(), b->pending.begin() + nt);
      b->pending.erase(b->pending.begin(), b->pending.begin() + nt);
      if (!b->pending.empty()) b->first_t = clk::now();
      lk.unlock();
      const int rc = launch(b, take);
      lk.lock();
      int slot_iters = 0;
      for (auto *q : take) {
        q->rc = rc;
        q->done = true;
        b->events.push_back(q->in);
        slot_iters += q->c->len;
      }
      b->stat[0] += 1;
      b->stat[1] += (double)take.size();
      b->stat[2] += slot_iters;
      b->stat[3] = std::max(b->stat[3], (double)take.size());
      b->launching = false;
      b->cv.notify_all();
    } else {
      b->cv.wait_until(lk, b->launching ? clk::now() + std::chrono::microseconds(20)
                                        : b->first_t + b->window);
    }
  }
  return p.rc;
}

// ====================================================================== C ABI
extern "C" int rbicg_batch_create(int32_t max_slots, double window_us, rbicg_batch *out) {
  if (!out) return rbicg_fail(RBICG_EINVAL, "null argument");
  if (max_slots < 1 || max_slots > RBICG_BATCH_SLOTS)
    return rbicg_fail(RBICG_EINVAL, "max_slots=%d out of range [1, %d]", max_slots, RBICG_BATCH_SLOTS);
  if (!(window_us >= 0) || window_us > 1e6) return rbicg_fail(RBICG_EINVAL, "window_us out of range");
  rbicg_batch b = new rbicg_batch_s();
  b->max_slots = max_slots;
  b->window = std::chrono::microseconds((long)window_us);
  for (int i = 0; i < NSTREAM; ++i)
    if (hipStreamCreateWithFlags(&b->sts[i], hipStreamNonBlocking) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipStreamDestroy(b->sts[j]);
      delete b;
      return rbicg_fail(RBICG_EHIP, "hipStreamCreate failed");
    }
  b->st = b->sts[0];
  *out = b;
  return RBICG_OK;
}

extern "C" int rbicg_batch_stats(rbicg_batch b, double *out) {
  if (!b || !out) return rbicg_fail(RBICG_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(b->mu);
  for (int i = 0; i < 6; ++i) out[i] = b->stat[i];
  return RBICG_OK;
}

extern "C" int rbicg_batch_use_graphs(rbicg_batch b, int32_t on) {
  if (!b) return rbicg_fail(RBICG_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(b->mu);
  while (b->launching) {  // not while a launch is being built
    lk.unlock();
    std::this_thread::yield();
    lk.lock();
  }
  b->graphs = on != 0;
  return RBICG_OK;
}

extern "C" int rbicg_batch_destroy(rbicg_batch b) {
  if (!b) return RBICG_OK;
  for (int i = 0; i < NSTREAM; ++i) (void)hipStreamSynchronize(b->sts[i]);
  for (int i = 0; i < NBUF; ++i) {
    if (b->host[i]) (void)hipHostFree(b->host[i]);
    if (b->dev[i]) (void)hipFree(b->dev[i]);
    if (b->used[i]) (void)hipEventDestroy(b->used[i]);
  }
  for (auto e : b->events) (void)hipEventDestroy(e);
  for (auto &kv : b->cap_sets) (void)hipGraphExecDestroy(kv.second.exec);
  for (int i = 0; i < NSTREAM; ++i) (void)hipStreamDestroy(b->sts[i]);
  delete b;
  return RBICG_OK;
}

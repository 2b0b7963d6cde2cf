// CPU stand-in for the HIP runtime and the kernel launchers, for running the
// library's host code (compile, validation, schedules, merged tables, the
// serving scheduler) without a GPU.  "Device" memory is host malloc; each
// launcher checks its launch against the design and touches the first and
// last element of every extent the real kernel reads or writes, so a
// host/kernel size disagreement faults here (or shows up under a sanitizer).
// No kernel arithmetic runs: outputs are placeholders.  Test infrastructure.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <map>
#include <set>
#include <thread>
#include <vector>

#include DP_KERNELS_H
#include DP_ABI_H

// dp_forward_static's device scratch lives in a HIP source the stand-in
// does not build; contexts only resolve its address.
namespace dp {
dp_status static_scratch_init(int) { return DP_OK; }
}  // namespace dp
extern "C" dp_status dp_forward_static(const dp_design *, const dp_params *, const float *,
                                       const float *, const float *, float *, float *, float *) {
  return DP_E_UNSUPPORTED;
}

// ---- stream capture model -------------------------------------------------
// A capture begins on one stream; another stream joins it by waiting on an
// event recorded in it (a fork) and must be waited on again, through an
// event recorded on it, before the capture ends (a join), or the end fails
// as unjoined.  Work enqueued on a capturing stream is recorded, not run:
// each launch's extents (every range the real kernel would touch) go into
// the graph, and every launch of the instantiated graph checks that each
// extent still lies inside a live allocation.  Calls the thread-local
// capture mode forbids while the calling thread captures (allocation, free,
// synchronization) abort, and so does waiting on an event whose last record
// belongs to an ended capture.
struct Extent {
  const void *p;
  size_t bytes;
  const char *what;
};
struct Capture {
  hipStream_t origin;
  std::thread::id thread;
  std::vector<Extent> extents;
  std::set<hipStream_t> members;  // origin and joined streams
  std::set<hipStream_t> forked;   // joined streams not yet joined back
  bool broken = false;
};
struct ihipStream_t { Capture *cap = nullptr; };
struct ihipEvent_t {
  Capture *cap = nullptr;   // the capture it was last recorded in (null: recorded outside)
  hipStream_t from = nullptr;
  bool stale = false;       // last recorded in a capture that has ended
};
struct ihipGraph { std::vector<Extent> extents; };
struct hipGraphExec { std::vector<Extent> extents; };

static std::mutex g_mu;
static std::map<const char *, size_t> g_live;  // allocation base -> bytes
static std::set<Capture *> g_caps;             // captures in progress
static std::set<hipEvent_t> g_events;
static long g_forks = 0, g_captures = 0, g_graph_launches = 0;

static void fatal(const char *msg) {
  std::fprintf(stderr, "STUB: %s\n", msg);
  std::abort();
}
static void note_alloc(void *p, size_t n) {
  std::lock_guard<std::mutex> l(g_mu);
  g_live[static_cast<const char *>(p)] = n;
}
static bool note_free(void *p) {
  std::lock_guard<std::mutex> l(g_mu);
  return g_live.erase(static_cast<const char *>(p)) == 1;
}
static bool is_live(const void *p, size_t bytes) {
  std::lock_guard<std::mutex> l(g_mu);
  const char *c = static_cast<const char *>(p);
  auto it = g_live.upper_bound(c);
  if (it == g_live.begin()) return false;
  --it;
  return c >= it->first && c + bytes <= it->first + it->second;
}
// Whether the calling thread is capturing (thread-local capture mode).
static bool thread_captures() {
  std::lock_guard<std::mutex> l(g_mu);
  for (Capture *c : g_caps)
    if (c->thread == std::this_thread::get_id()) return true;
  return false;
}
static void end_capture(Capture *c) {
  {
    std::lock_guard<std::mutex> l(g_mu);
    g_caps.erase(c);
    for (hipEvent_t e : g_events)
      if (e->cap == c) {
        e->cap = nullptr;
        e->stale = true;
      }
  }
  for (hipStream_t m : c->members) m->cap = nullptr;
  delete c;
}

// Recording target of the launch being made (null: run, i.e. touch memory).
static thread_local Capture *g_rec = nullptr;
struct Scope {
  Capture *prev;
  explicit Scope(hipStream_t s) : prev(g_rec) { g_rec = s ? s->cap : nullptr; }
  ~Scope() { g_rec = prev; }
};

extern "C" {
// Counts of what the capture model saw: captures, forks into them, graph
// launches (read by the host-logic scenarios).
void stub_capture_counts(long *out) {
  out[0] = g_captures;
  out[1] = g_forks;
  out[2] = g_graph_launches;
}
hipError_t hipMalloc(void **ptr, size_t size) {
  if (thread_captures()) fatal("hipMalloc while this thread captures a stream");
  *ptr = std::malloc(size ? size : 1);
  note_alloc(*ptr, size ? size : 1);
  return hipSuccess;
}
hipError_t hipFree(void *ptr) {
  if (!ptr) return hipSuccess;
  if (thread_captures()) fatal("hipFree while this thread captures a stream");
  if (!note_free(ptr)) { std::fprintf(stderr, "STUB: hipFree of unknown %p\n", ptr); std::abort(); }
  std::free(ptr);
  return hipSuccess;
}
hipError_t hipHostMalloc(void **ptr, size_t size, unsigned int) { return hipMalloc(ptr, size); }
hipError_t hipHostFree(void *ptr) { return hipFree(ptr); }
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t s) {
  if (s && s->cap) {
    s->cap->extents.push_back({dst, n, "copy destination"});
    s->cap->extents.push_back({src, n, "copy source"});
    return hipSuccess;
  }
  if (n) std::memmove(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind) {
  if (thread_captures()) fatal("hipMemcpy while this thread captures a stream");
  if (n) std::memmove(dst, src, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (s && s->cap) fatal("hipStreamSynchronize of a capturing stream");
  if (thread_captures()) fatal("hipStreamSynchronize while this thread captures a stream");
  return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "stub error"; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) {
  *e = new ihipEvent_t();
  std::lock_guard<std::mutex> l(g_mu);
  g_events.insert(*e);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  {
    std::lock_guard<std::mutex> l(g_mu);
    g_events.erase(e);
  }
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  e->cap = s ? s->cap : nullptr;
  e->from = s;
  e->stale = false;
  return hipSuccess;
}
static void check_usable(hipEvent_t e, const char *what) {
  if (e->cap) {
    std::fprintf(stderr, "STUB: %s of an event recorded in a capture in progress\n", what);
    std::abort();
  }
  if (e->stale) {
    std::fprintf(stderr, "STUB: %s of an event last recorded in an ended capture\n", what);
    std::abort();
  }
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  check_usable(e, "hipEventSynchronize");
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  check_usable(e, "hipEventQuery");
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  check_usable(a, "hipEventElapsedTime");
  check_usable(b, "hipEventElapsedTime");
  *ms = 0.001f;
  return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t *s) { *s = new ihipStream_t(); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = new ihipStream_t(); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) {
  if (s && s->cap) fatal("hipStreamDestroy of a capturing stream");
  delete s;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  Capture *c = e->cap;
  Capture *sc = s ? s->cap : nullptr;
  if (c) {
    if (!s) fatal("the null stream waits on an event of a capture");
    if (sc && sc != c) fatal("a stream of one capture waits on an event of another");
    if (!sc) {  // a fork: s joins the capture
      ++g_forks;
      s->cap = c;
      c->members.insert(s);
      c->forked.insert(s);
    } else if (e->from != s) {
      c->forked.erase(e->from);  // a join of the branch the event was recorded on
    }
    return hipSuccess;
  }
  if (sc) fatal("a capturing stream waits on an event recorded outside the capture");
  if (e->stale) fatal("a stream waits on an event last recorded in an ended capture");
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s) return hipErrorInvalidValue;
  if (s->cap) fatal("hipStreamBeginCapture on a stream that already captures");
  ++g_captures;
  auto *c = new Capture();
  c->origin = s;
  c->thread = std::this_thread::get_id();
  c->members.insert(s);
  s->cap = c;
  std::lock_guard<std::mutex> l(g_mu);
  g_caps.insert(c);
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
  Capture *c = s ? s->cap : nullptr;
  if (!c || c->origin != s) fatal("hipStreamEndCapture on a stream that did not begin a capture");
  const bool unjoined = !c->forked.empty();
  auto *graph = new ihipGraph();
  graph->extents = c->extents;
  end_capture(c);
  if (unjoined) {
    delete graph;
    *g = nullptr;
    std::fprintf(stderr, "STUB: capture ended with a forked stream not joined back\n");
    return hipErrorStreamCaptureUnjoined;
  }
  *g = graph;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
  *x = new hipGraphExec();
  (*x)->extents = g->extents;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t x) { delete x; return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  if (s && s->cap) {
    s->cap->extents.insert(s->cap->extents.end(), x->extents.begin(), x->extents.end());
    return hipSuccess;
  }
  ++g_graph_launches;
  for (const Extent &e : x->extents)
    if (e.bytes && !is_live(e.p, e.bytes)) {
      std::fprintf(stderr, "STUB: graph launch touches %zu bytes at %p (%s) outside any live "
                           "allocation\n", e.bytes, e.p, e.what);
      std::abort();
    }
  return hipSuccess;
}
}

// ---- launchers: touch the extents ------------------------------------------
#define CONTRIB_ELEMS(g) n_edges_of(g)
namespace {
template <class T>
void rd(const T *p, int64_t n) {
  if (n <= 0) return;
  if (!p) { std::fprintf(stderr, "STUB: null read of %lld\n", (long long)n); std::abort(); }
  if (g_rec) {  // captured: checked when the graph is launched
    g_rec->extents.push_back({p, (size_t)n * sizeof(T), "kernel read"});
    return;
  }
  volatile T a = p[0]; volatile T b = p[n - 1]; (void)a; (void)b;
}
template <class T>
void wr(T *p, int64_t n) {
  if (n <= 0) return;
  if (!p) { std::fprintf(stderr, "STUB: null write of %lld\n", (long long)n); std::abort(); }
  if (g_rec) {
    g_rec->extents.push_back({p, (size_t)n * sizeof(T), "kernel write"});
    return;
  }
  std::memset((void *)&p[0], 0, sizeof(T));
  std::memset((void *)&p[n - 1], 0, sizeof(T));
}
int64_t n_edges_of(const dp::GraphView &g) { return g.rev_ptr[g.n_nets]; }
void rd_graph(const dp::GraphView &g, int32_t g0, int32_t n, bool cells) {
  rd(g.op + g0, n);
  for (int k = 0; k < g.pins; ++k) rd(g.in + (int64_t)k * g.G + g0, n);
  for (int k = 0; k < g.pins; ++k) rd(g.slot + (int64_t)k * g.G + g0, n);
  if (g0 < 0 || n < 0 || g0 + n > g.G) { std::fprintf(stderr, "STUB: range out of G\n"); std::abort(); }
  for (int32_t i = g0; i < g0 + n; ++i) {
    const bool is_cell = g.op[i] >= dp::kCellBase;
    if (is_cell != cells) { std::fprintf(stderr, "STUB: gate %d kind mismatch\n", i); std::abort(); }
    if (is_cell) {
      const int c = g.op[i] - dp::kCellBase;
      const int off = g.cell[3 * c], len = g.cell[3 * c + 1], nin = g.cell[3 * c + 2];
      rd(g.code + off, len);
      rd(g.tt + c, 1);
      if (nin > g.pins || len > dp::kCellMaxCode) { std::fprintf(stderr, "STUB: cell\n"); std::abort(); }
    }
  }
}
}  // namespace

namespace dp {
constexpr int32_t kPowerChunk = 2048, kSlabNets = 2048;

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t stream_) {
  Scope sc_(stream_);
  for (int64_t i = 0; i < n; ++i) p[i] = v;
  return hipSuccess;
}
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t stream_) {
  Scope sc_(stream_);
  for (int64_t i = 0; i < n; ++i) p[i] = v;
  return hipSuccess;
}
hipError_t launch_load_pi(const float *p, float *sp, int32_t n_pi, int32_t B, hipStream_t stream_) {
  Scope sc_(stream_);
  rd(p, (int64_t)n_pi * B);
  wr(sp, (int64_t)n_pi * B);
  return hipSuccess;
}
hipError_t launch_check_range(const float *v, int64_t n, float lo, float hi, int32_t *bad,
                              hipStream_t stream_) {
  Scope sc_(stream_);
  int32_t b = 0;
  for (int64_t i = 0; i < n; ++i)
    if (!(v[i] >= lo && v[i] <= hi)) b = 1;
  *bad = b;
  return hipSuccess;
}
hipError_t launch_gather_nets_f32(const float *src, const int32_t *int2ext, float *dst,
                                  int32_t n_nets, hipStream_t stream_) {
  Scope sc_(stream_);
  for (int32_t i = 0; i < n_nets; ++i) dst[i] = src[int2ext[i]];
  return hipSuccess;
}
hipError_t launch_import_cols_f32(const float *src, const int32_t *int2ext, float *dst,
                                  int32_t n_nets, int32_t B, hipStream_t stream_) {
  Scope sc_(stream_);
  for (int32_t i = 0; i < n_nets; ++i)
    for (int32_t b = 0; b < B; ++b) dst[(int64_t)i * B + b] = src[(int64_t)b * n_nets + int2ext[i]];
  return hipSuccess;
}
hipError_t launch_import_sizes(const float *src, const int32_t *int2ext, float *dst, int32_t n_pi,
                               int32_t G, int32_t S, hipStream_t stream_) {
  Scope sc_(stream_);
  rd(int2ext, n_pi + G);
  rd(src, (int64_t)S * G);
  wr(dst, (int64_t)S * G);
  return hipSuccess;
}
hipError_t launch_sp_level(const GraphView &g, const SpLevel &lv, bool cells, hipStream_t stream_) {
  Scope sc_(stream_);
  rd_graph(g, lv.g0, lv.n, cells);
  wr(lv.sp + (int64_t)(g.n_pi + lv.g0) * lv.B, (int64_t)lv.n * lv.B);
  return hipSuccess;
}
hipError_t launch_sp_pair(const GraphView &g, const SpLevel &a, const SpLevel &b, hipStream_t stream_) {
  Scope sc_(stream_);
  if (a.B != b.B || a.sp != b.sp || b.g0 != a.g0 + a.n) fatal("level pair not adjacent");
  rd_graph(g, a.g0, a.n, false);
  rd_graph(g, b.g0, b.n, false);
  // every pin of the second level is stored before the launch or driven by
  // the first level, whose gates read only nets stored before the launch
  static const int kAr[9] = {1, 1, 2, 2, 2, 2, 2, 3, 3};
  const int32_t lo = g.n_pi + a.g0, hi = lo + a.n;
  for (int32_t i = a.g0; i < a.g0 + a.n; ++i)
    for (int k = 0; k < kAr[g.op[i]]; ++k)
      if (g.in[(int64_t)k * g.G + i] >= lo) fatal("first level of a pair reads its own level");
  for (int32_t i = b.g0; i < b.g0 + b.n; ++i)
    for (int k = 0; k < kAr[g.op[i]]; ++k)
      if (g.in[(int64_t)k * g.G + i] >= hi) fatal("second level of a pair reads its own level");
  wr(a.sp + (int64_t)(g.n_pi + a.g0) * a.B, ((int64_t)a.n + b.n) * a.B);
  return hipSuccess;
}
hipError_t launch_markov_words(const float *sp, const float *tau, const int32_t *stream,
                               int32_t n_pi, int32_t B, int64_t T, uint64_t, uint64_t *out,
                               hipStream_t stream_) {
  Scope sc_(stream_);
  rd(sp, (int64_t)n_pi * B);
  rd(tau, (int64_t)n_pi * B);
  if (stream) {
    rd(stream, n_pi);
    for (int32_t i = 0; i < n_pi; ++i)
      if (stream[i] < 0 || stream[i] >= n_pi) { std::fprintf(stderr, "STUB: stream\n"); std::abort(); }
  }
  wr(out, (int64_t)n_pi * B * T);
  return hipSuccess;
}
hipError_t launch_stimulus(const GraphView &g, const ChunkView &c, const CountView &cnt,
                           const float *p_col, const uint64_t *stim, int64_t T,
                           const int32_t *stream, uint64_t, const SimTune &, hipStream_t stream_) {
  Scope sc_(stream_);
  if (stream) rd(stream, g.n_pi);
  if (c.n_cols < 1 || cnt.col < 0 || cnt.col + c.n_cols > cnt.B) {
    std::fprintf(stderr, "STUB: stimulus columns out of range\n");
    std::abort();
  }
  for (int32_t k = 0; k < c.n_cols; ++k) wr(c.W + k * c.col_stride, (int64_t)g.n_pi * c.pitch);
  rd(p_col, (int64_t)g.n_pi * cnt.B);
  if (stim) rd(stim, (int64_t)c.n_cols * g.n_pi * T);
  wr(cnt.ones, (int64_t)g.n_pi * cnt.B);
  wr(cnt.tog, (int64_t)g.n_pi * cnt.B);
  if (c.u_hi > c.pitch || c.u_lo < 0 || 2 * c.pairs > c.pitch) {
    std::fprintf(stderr, "STUB: chunk view out of pitch\n");
    std::abort();
  }
  return hipSuccess;
}
hipError_t launch_sim_level(const GraphView &g, const ChunkView &c, const CountView &cnt,
                            int32_t g0, int32_t n, const SpLevel *sp, bool cells,
                            const SimTune &, hipStream_t stream_, int cell_inputs) {
  Scope sc_(stream_);
  rd_graph(g, g0, n, cells);
  if (sp) rd_graph(g, sp->g0, sp->n, cells);  // the fused SP: gates of the same kind
  if (cells)  // every cell of the range within the instance's input count
    for (int32_t i = g0; i < g0 + n; ++i)
      if (g.cell[3 * (g.op[i] - dp::kCellBase) + 2] > cell_inputs)
        fatal("library cell wider than its simulation launch");
  if (c.n_cols < 1 || cnt.col < 0 || cnt.col + c.n_cols > cnt.B) {
    std::fprintf(stderr, "STUB: simulation columns out of range\n");
    std::abort();
  }
  for (int32_t k = 0; k < c.n_cols; ++k) {
    rd(c.W + k * c.col_stride, (int64_t)g.n_nets * c.pitch);  // fan-in rows anywhere below
    wr(c.W + k * c.col_stride + (int64_t)(g.n_pi + g0) * c.pitch, (int64_t)n * c.pitch);
  }
  wr(cnt.ones + (int64_t)(g.n_pi + g0) * cnt.B, (int64_t)n * cnt.B);
  wr(cnt.tog + (int64_t)(g.n_pi + g0) * cnt.B, (int64_t)n * cnt.B);
  if (sp) wr(sp->sp + (int64_t)(g.n_pi + g0) * sp->B, (int64_t)n * sp->B);
  return hipSuccess;
}
hipError_t launch_export(const ExportArgs &a, hipStream_t stream_) {
  Scope sc_(stream_);
  const int64_t nb = (int64_t)a.n_nets * a.B;
  rd(a.sp, nb);
  if (a.beta) rd(a.beta, nb);
  rd(a.int2ext, a.n_nets);
  if (a.o_sp) wr(a.o_sp, nb);
  if (a.o_tr) wr(a.o_tr, nb);
  if (a.o_sp_acc) { rd(a.ones, nb); wr(a.o_sp_acc, nb); }
  if (a.o_tr_acc) { rd(a.tog, nb); wr(a.o_tr_acc, nb); }
  if (a.o_beta) wr(a.o_beta, nb);
  if (a.o_tr_hyb) wr(a.o_tr_hyb, nb);
  if (a.o_ones) { rd(a.ones, nb); wr(a.o_ones, nb); }
  if (a.o_tog) { rd(a.tog, nb); wr(a.o_tog, nb); }
  return hipSuccess;
}
int32_t power_chunks(int32_t n_nets) {
  return n_nets <= 0 ? 1 : (n_nets + kPowerChunk - 1) / kPowerChunk;
}
int32_t power_partial_doubles(int32_t n_nets, int32_t B, int32_t S, int32_t paired) {
  const int64_t cols = (int64_t)B * ((S > 0 && !paired) ? S : 1);
  int64_t slabs = power_chunks(n_nets);
  if (S > 0 && !paired) slabs = std::max<int64_t>(slabs, (n_nets + kSlabNets - 1) / kSlabNets);
  return (int32_t)(slabs * cols);
}
hipError_t launch_power(const PowerArgs &a, hipStream_t stream_) {
  Scope sc_(stream_);
  const int64_t nb = (int64_t)a.n_nets * a.B;
  rd(a.sp, nb);
  if (a.mode == 1) {  // hybrid: toggle counts in, beta out
    rd(a.tog, nb);
    if (!a.beta) fatal("hybrid power without its beta output");
    wr(a.beta, nb);
  }
  if (a.beta_frozen) rd(a.beta_frozen, a.beta_shared ? a.n_nets : nb);
  rd(a.cap, a.n_nets);
  if (a.S > 0 && a.size) rd(a.size, (int64_t)a.S * a.G);
  if (a.n_chunks != power_chunks(a.n_nets)) fatal("power chunk count");
  wr(a.partial, power_partial_doubles(a.n_nets, a.B, a.S, a.paired));
  const int64_t Sp = (a.S > 0 && !a.paired) ? a.S : 1;
  wr(a.power, a.B * Sp);
  return hipSuccess;
}
constexpr int32_t kNoHeavyCheck = -1;  // a caller of the stand-in that passes no list
hipError_t launch_bwd_level(const GraphView &g, const BwdArgs &a, int32_t g0, int32_t n,
                            bool cells, hipStream_t stream_, const int32_t *heavy,
                            int32_t n_heavy) {
  Scope sc_(stream_);
  rd_graph(g, g0, n, cells);
  // the heavy list: every gate of the range whose fan-out range is longer
  // than kHeavyPull, ascending, and nothing else
  if ((n_heavy < 0 && n_heavy != kNoHeavyCheck) || (n_heavy > 0 && !heavy)) fatal("heavy list");
  rd(heavy, n_heavy);
  if (!cells && n_heavy != kNoHeavyCheck) {
    int32_t k = 0;
    for (int32_t gi = g0; gi < g0 + n; ++gi) {
      const int32_t out = g.n_pi + gi;
      if (g.rev_ptr[out + 1] - g.rev_ptr[out] <= dp::kHeavyPull) continue;
      if (k >= n_heavy || heavy[k] != gi) fatal("heavy list misses a gate");
      ++k;
    }
    if (k != n_heavy) fatal("heavy list holds a gate it should not");
  }
  rd(a.sp, (int64_t)g.n_nets * a.B);
  rd(a.cap, g.n_nets);
  if (a.size) rd(a.size, (int64_t)(a.S > 0 ? a.S : a.B) * a.G);
  if (a.w) rd(a.w, (int64_t)a.C);
  wr(a.contrib, CONTRIB_ELEMS(g) * a.C);
  if (a.lam) wr(a.lam, (int64_t)g.n_nets * a.C);
  if (a.beta) rd(a.beta, a.beta_shared ? (int64_t)g.n_nets : (int64_t)g.n_nets * a.B);
  if ((int64_t)a.C > (int64_t)a.B * a.cdiv) { std::fprintf(stderr, "STUB: C > B*cdiv\n"); std::abort(); }
  return hipSuccess;
}
hipError_t launch_bwd_pi(const GraphView &g, const BwdArgs &a, float *out, hipStream_t stream_,
                         const int32_t *heavy, int32_t n_heavy) {
  Scope sc_(stream_);
  if ((n_heavy < 0 && n_heavy != kNoHeavyCheck) || (n_heavy > 0 && !heavy)) fatal("heavy PI list");
  rd(heavy, n_heavy);
  if (n_heavy != kNoHeavyCheck) {  // every PI with a long fan-out range, ascending, no other
    int32_t k = 0;
    for (int32_t i = 0; i < g.n_pi; ++i) {
      if (g.rev_ptr[i + 1] - g.rev_ptr[i] <= dp::kHeavyPull) continue;
      if (k >= n_heavy || heavy[k] != i) fatal("heavy PI list misses a PI");
      ++k;
    }
    if (k != n_heavy) fatal("heavy PI list holds a PI it should not");
  }
  if (a.fixed) rd(a.fixed, g.n_pi);
  rd(a.contrib, CONTRIB_ELEMS(g) * a.C);
  wr(out, (int64_t)a.C * g.n_pi);
  return hipSuccess;
}
hipError_t launch_sp_persistent(const GraphView &g, const SpLevel &lv, const int32_t *level_ptr,
                                int32_t depth, int64_t, GridBarrier bar, hipStream_t stream_) {
  Scope sc_(stream_);
  rd(level_ptr, depth + 2);
  wr(bar.words, kBarrierWords);
  rd(bar.words + kBarrierReport, 1);
  wr(lv.sp, (int64_t)g.n_nets * lv.B);
  return hipSuccess;
}
hipError_t launch_bwd_persistent(const GraphView &g, const BwdArgs &a, const int32_t *level_ptr,
                                 int32_t depth, int64_t, float *pi_out, GridBarrier bar,
                                 hipStream_t s) {
  Scope sc_(s);
  rd(level_ptr, depth + 2);
  wr(bar.words, kBarrierWords);
  rd(bar.words + kBarrierReport, 1);
  return launch_bwd_pi(g, a, pi_out, s, nullptr, kNoHeavyCheck);  // its own PI pass
}
hipError_t launch_sp_multi(const SpSeg *segs, int32_t n_segs, uint32_t blocks, bool cells,
                           hipStream_t st) {
  Scope sc_(st);
  for (int32_t k = 0; k < n_segs; ++k) {
    const uint32_t b0 = segs[k].block0, b1 = k + 1 < n_segs ? segs[k + 1].block0 : blocks;
    const int64_t items = ((int64_t)segs[k].lv.n + segs[k].lv2.n) * segs[k].lv.B;
    if (b1 < b0 || (int64_t)(b1 - b0) * kMergedBlock < items) {
      std::fprintf(stderr, "STUB: sp segment %d too small\n", k);
      std::abort();
    }
    if (segs[k].lv2.n > 0) {  // a pair: the single-design pair launch's checks
      if (cells) fatal("a paired segment in a library-cell launch");
      launch_sp_pair(segs[k].g, segs[k].lv, segs[k].lv2, st);
    } else {
      launch_sp_level(segs[k].g, segs[k].lv, cells, st);
    }
  }
  return hipSuccess;
}
hipError_t launch_bwd_multi(const BwdSeg *segs, int32_t n_segs, uint32_t blocks, bool cells,
                            hipStream_t st) {
  Scope sc_(st);
  for (int32_t k = 0; k < n_segs; ++k) {
    const uint32_t b0 = segs[k].block0, b1 = k + 1 < n_segs ? segs[k + 1].block0 : blocks;
    if (b1 < b0 || (int64_t)(b1 - b0) * kMergedBlock < (int64_t)segs[k].n * segs[k].a.C) {
      std::fprintf(stderr, "STUB: bwd segment %d too small\n", k);
      std::abort();
    }
    // merged launches pull every gate in its own item (no heavy list)
    launch_bwd_level(segs[k].g, segs[k].a, segs[k].g0, segs[k].n, cells, st, nullptr,
                     kNoHeavyCheck);
  }
  return hipSuccess;
}
hipError_t launch_grad_lambda_export(const float *lam, const float *sp, const int32_t *int2ext,
                                     int32_t n_pi, int32_t n_nets, int32_t B, int32_t C,
                                     int32_t, float, float *lam_out, float *score, hipStream_t stream_) {
  Scope sc_(stream_);
  rd(lam, (int64_t)n_nets * C);
  rd(sp, (int64_t)n_nets * B);
  rd(int2ext, n_nets);
  if (lam_out) wr(lam_out, (int64_t)n_nets * C);
  if (score) wr(score, (int64_t)(n_nets - n_pi) * C);
  return hipSuccess;
}
hipError_t launch_virus_step(float *sp, const float *grad, float, int32_t n_pi, int32_t B, hipStream_t stream_) {
  Scope sc_(stream_);
  wr(sp, (int64_t)n_pi * B);
  rd(grad, (int64_t)n_pi * B);
  return hipSuccess;
}
hipError_t launch_virus_vectors(const float *sp, uint64_t *stim, uint8_t *v0, float *p_out,
                                int32_t n_pi, int32_t B, hipStream_t stream_) {
  Scope sc_(stream_);
  rd(sp, (int64_t)n_pi * B);
  wr(stim, (int64_t)n_pi * B * 2);
  wr(v0, (int64_t)n_pi * B);
  if (p_out) wr(p_out, (int64_t)n_pi * B);
  return hipSuccess;
}
hipError_t launch_virus_power(const uint32_t *tog, const float *cap, int32_t n_nets, int32_t B,
                              double *out, hipStream_t stream_) {
  Scope sc_(stream_);
  rd(tog, (int64_t)n_nets * B);
  rd(cap, n_nets);
  wr(out, B);
  return hipSuccess;
}
hipError_t launch_grad_export(const GradExportArgs &a, hipStream_t stream_) {
  Scope sc_(stream_);
  const int64_t nb = (int64_t)a.n_nets * a.B;
  rd(a.sp, nb);
  if (a.beta) rd(a.beta, a.beta_shared ? a.n_nets : nb);
  rd(a.cap, a.n_nets);
  rd(a.int2ext, a.n_nets);
  if (a.dcap) wr(a.dcap, a.n_nets);
  if (a.dsize) wr(a.dsize, (int64_t)a.S * a.G);
  return hipSuccess;
}
}  // namespace dp

// Host-only stand-in for the HIP runtime calls that libidp_dg makes, so that
// the library's host code (handles, batches, graphs, staging) can run under
// AddressSanitizer on a machine without a GPU.  Kernels do not run.  Work on
// a stream is a queue of pending operations that completes only when the
// host synchronises, queries an event (one operation per query) or, every
// seventh call, by itself; the stand-in aborts on API misuse that the real
// runtime would turn into memory corruption: destroying a graph exec with a
// launch still pending, freeing memory twice, freeing pinned memory or
// changing it while a copy from it is pending, using destroyed handles.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cstdint>
#include <map>
#include <set>
#include <vector>
#include <deque>
#include <string>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorNotReady = 600 };
struct dim3 { unsigned x, y, z; };

#define FAIL(...) do { fprintf(stderr, "MOCK ERROR: " __VA_ARGS__); fprintf(stderr, "\n"); abort(); } while (0)

struct Op {
  int kind;            // 0 kernel, 1 memcpy, 2 event record, 3 graph launch, 4 memset
  uint64_t seq;
  const void* hsrc; size_t bytes; uint64_t sum;   // memcpy from host: checksum at enqueue
  void* exec;
  void* event;
};
struct Stream { std::deque<Op> q; uint64_t next = 1, done = 0; bool live = true; void* capture = nullptr; };
struct Event { bool live = true; Stream* s = nullptr; uint64_t seq = 0; bool recorded = false; };
struct Node { const void* func; };
struct Graph { bool live = true; std::vector<Node> nodes; };
struct Exec { bool live = true; Graph* g; int pending = 0; };

static std::map<void*, size_t> g_dev, g_host;
static std::set<Stream*> g_streams;
static std::set<Event*> g_events;
static std::set<Graph*> g_graphs;
static std::set<Exec*> g_execs;
static Stream g_null;
static uint64_t g_ops = 0;

static uint64_t checksum(const void* p, size_t n) {
  const unsigned char* c = (const unsigned char*)p; uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}
static Stream* S(void* s) {
  if (!s) return &g_null;
  Stream* st = (Stream*)s;
  if (!g_streams.count(st) || !st->live) FAIL("use of a destroyed or unknown stream %p", s);
  return st;
}
static void complete(Stream* st, Op& op) {
  if (op.kind == 1 && op.hsrc) {
    if (checksum(op.hsrc, op.bytes) != op.sum) FAIL("host source of an async copy changed before the copy ran");
  }
  if (op.kind == 3) {
    Exec* e = (Exec*)op.exec;
    if (!g_execs.count(e) || !e->live) FAIL("graph exec destroyed while its launch was pending");
    e->pending--;
  }
  st->done = op.seq;
}
static void drain(Stream* st, uint64_t upto) {
  while (!st->q.empty() && st->q.front().seq <= upto) { Op op = st->q.front(); st->q.pop_front(); complete(st, op); }
}
static uint64_t push(Stream* st, Op op) {
  op.seq = st->next++;
  st->q.push_back(op);
  // background progress: every 7th call completes the oldest op of this stream
  if (++g_ops % 7 == 0 && !st->q.empty()) { Op o = st->q.front(); st->q.pop_front(); complete(st, o); }
  return op.seq;
}
static bool pending_host_read(const void* p, size_t n) {
  auto chk = [&](Stream* st) {
    for (auto& op : st->q) if (op.kind == 1 && op.hsrc && (const char*)op.hsrc < (const char*)p + n && (const char*)p < (const char*)op.hsrc + op.bytes) return true;
    return false; };
  if (chk(&g_null)) return true;
  for (auto* st : g_streams) if (st->live && chk(st)) return true;
  return false;
}

extern "C" {
const char* hipGetErrorString(hipError_t) { return "mock error"; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipMalloc(void** p, size_t n) {
  *p = aligned_alloc(256, ((n + 255) / 256) * 256 + 256); memset(*p, 0, n); g_dev[*p] = n; return hipSuccess; }
hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  if (!g_dev.count(p)) FAIL("hipFree of %p: not a live device allocation", p);
  g_dev.erase(p); free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
  *p = aligned_alloc(256, ((n + 255) / 256) * 256 + 256); g_host[*p] = n; return hipSuccess; }
hipError_t hipHostFree(void* p) {
  if (!p) return hipSuccess;
  if (!g_host.count(p)) FAIL("hipHostFree of %p: not a live pinned allocation", p);
  if (pending_host_read(p, g_host[p])) FAIL("hipHostFree while an async copy from it is pending");
  g_host.erase(p); free(p); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, int kind, void* stream) {
  Stream* st = S(stream);
  bool from_host = false;
  for (auto& kv : g_host) if ((const char*)s >= (const char*)kv.first && (const char*)s + n <= (const char*)kv.first + kv.second) from_host = true;
  memcpy(d, s, n);   // data moves now; a later change of the source is detected at completion
  Op op{}; op.kind = 1; op.hsrc = from_host ? s : nullptr; op.bytes = n; op.sum = from_host ? checksum(s, n) : 0;
  if (st->capture) FAIL("memcpy recorded into a captured graph");
  push(st, op); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, void* stream) {
  Stream* st = S(stream); if (st->capture) FAIL("memset recorded into a captured graph");
  memset(d, v, n); Op op{}; op.kind = 4; push(st, op); return hipSuccess; }
hipError_t hipMemset(void* d, int v, size_t n) { memset(d, v, n); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(void** s, unsigned) { Stream* st = new Stream; g_streams.insert(st); *s = st; return hipSuccess; }
hipError_t hipStreamDestroy(void* s) { Stream* st = S(s); drain(st, ~0ull); st->live = false; return hipSuccess; }
hipError_t hipStreamSynchronize(void* s) { Stream* st = S(s); drain(st, ~0ull); return hipSuccess; }
hipError_t hipDeviceSynchronize() {
  drain(&g_null, ~0ull);
  for (auto* st : g_streams) if (st->live) drain(st, ~0ull);
  return hipSuccess; }
hipError_t hipEventCreateWithFlags(void** e, unsigned) { Event* ev = new Event; g_events.insert(ev); *e = ev; return hipSuccess; }
static Event* E(void* e) { Event* ev = (Event*)e; if (!g_events.count(ev) || !ev->live) FAIL("use of a destroyed or unknown event %p", e); return ev; }
hipError_t hipEventRecord(void* e, void* s) {
  Event* ev = E(e); Stream* st = S(s); if (st->capture) FAIL("event recorded into a capture");
  Op op{}; op.kind = 2; op.event = ev; ev->s = st; ev->seq = push(st, op); ev->recorded = true; return hipSuccess; }
hipError_t hipEventSynchronize(void* e) { Event* ev = E(e); if (ev->recorded) drain(ev->s, ev->seq); return hipSuccess; }
hipError_t hipEventQuery(void* e) {
  Event* ev = E(e); if (!ev->recorded || ev->s->done >= ev->seq) return hipSuccess;
  // one op of progress per query
  if (!ev->s->q.empty()) { Op o = ev->s->q.front(); ev->s->q.pop_front(); complete(ev->s, o); }
  return ev->s->done >= ev->seq ? hipSuccess : hipErrorNotReady; }
hipError_t hipEventDestroy(void* e) { Event* ev = E(e); ev->live = false; return hipSuccess; }
hipError_t hipEventCreate(void** e) { return hipEventCreateWithFlags(e, 0); }
// both events must have run: the elapsed time is a stand-in (no clock)
hipError_t hipEventElapsedTime(float* ms, void* a, void* b) {
  Event* ea = E(a); Event* eb = E(b);
  if (!ea->recorded || !eb->recorded || ea->s->done < ea->seq || eb->s->done < eb->seq)
    FAIL("elapsed time of events that have not completed");
  *ms = (float)(eb->seq - ea->seq); return hipSuccess; }
hipError_t hipGraphCreate(void** g, unsigned) { Graph* gr = new Graph; g_graphs.insert(gr); *g = gr; return hipSuccess; }
static Graph* G(void* g) { Graph* gr = (Graph*)g; if (!g_graphs.count(gr) || !gr->live) FAIL("use of a destroyed or unknown graph %p", g); return gr; }
// hipKernelNodeParams layout: dim3 blockDim; void** extra; void* func; dim3 gridDim; void** kernelParams; unsigned sharedMemBytes
struct hipKernelNodeParamsM { dim3 blockDim; void** extra; void* func; dim3 gridDim; void** kernelParams; unsigned sharedMemBytes; };
hipError_t hipGraphAddKernelNode(void** node, void* g, void* const* deps, size_t ndeps, const hipKernelNodeParamsM* kp) {
  Graph* gr = G(g);
  if (!kp || !kp->func || !kp->kernelParams) FAIL("kernel node without function or parameters");
  for (size_t i = 0; i < ndeps; ++i) { size_t idx = (size_t)deps[i] - 1; if (idx >= gr->nodes.size()) FAIL("dependency on a node of another graph"); }
  Node nd; nd.func = kp->func;
  gr->nodes.push_back(nd); *node = (void*)(uintptr_t)gr->nodes.size(); return hipSuccess; }
hipError_t hipGraphInstantiate(void** ex, void* g, void*, char*, size_t) {
  Graph* gr = G(g); Exec* e = new Exec; e->g = gr; g_execs.insert(e); *ex = e; return hipSuccess; }
hipError_t hipGraphLaunch(void* ex, void* s) {
  Exec* e = (Exec*)ex; if (!g_execs.count(e) || !e->live) FAIL("launch of a destroyed graph exec");
  Stream* st = S(s); Op op{}; op.kind = 3; op.exec = e; e->pending++; push(st, op); return hipSuccess; }
hipError_t hipGraphExecDestroy(void* ex) {
  Exec* e = (Exec*)ex; if (!g_execs.count(e) || !e->live) FAIL("double destroy of a graph exec");
  if (e->pending) FAIL("graph exec destroyed with %d launch(es) still pending", e->pending);
  e->live = false; return hipSuccess; }
hipError_t hipGraphDestroy(void* g) { Graph* gr = G(g); gr->live = false; return hipSuccess; }
hipError_t hipStreamBeginCapture(void* s, int) { Stream* st = S(s); st->capture = new Graph; g_graphs.insert((Graph*)st->capture); return hipSuccess; }
hipError_t hipStreamEndCapture(void* s, void** g) { Stream* st = S(s); *g = st->capture; st->capture = nullptr; return hipSuccess; }
static dim3 g_grid, g_block; static size_t g_shm; static void* g_cfg_stream;
unsigned __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shm, void* stream) { g_grid = grid; g_block = block; g_shm = shm; g_cfg_stream = stream; return 0; }
hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shm, void** stream) { *grid = g_grid; *block = g_block; *shm = g_shm; *stream = g_cfg_stream; return hipSuccess; }
hipError_t hipLaunchKernel(const void* f, dim3 grid, dim3 block, void** args, size_t, void* stream) {
  if (!f || !args) FAIL("kernel launch without function or args");
  if (grid.x == 0 || block.x == 0 || block.x > 1024) FAIL("bad launch shape %u x %u", grid.x, block.x);
  Stream* st = S(stream);
  if (st->capture) { Node nd; nd.func = f; ((Graph*)st->capture)->nodes.push_back(nd); return hipSuccess; }
  Op op{}; op.kind = 0; push(st, op); return hipSuccess; }
void** __hipRegisterFatBinary(const void*) { static void* h; return &h; }
void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned, void*, void*, void*, void*, int*) {}
void __hipRegisterVar(void**, void*, char*, const char*, int, size_t, int, int) {}
// a device symbol's "address": a host buffer standing in for it (the
// library only passes it to kernels, which do not run here)
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  static char stand_in[4096];
  if (!p || !sym) return hipErrorInvalidValue;
  *p = stand_in;
  return hipSuccess;
}
void __hipUnregisterFatBinary(void**) {}
// report what is still alive at exit
void mock_report() {
  size_t d = g_dev.size(), h = g_host.size(); int ex = 0; for (auto* e : g_execs) ex += e->live;
  fprintf(stderr, "mock: live device allocations %zu, pinned %zu, graph execs %d\n", d, h, ex);
}
}

// roctx ranges of the library's entry points: no tool attached
extern "C" int roctxRangePushA(const char*) { return 0; }
extern "C" int roctxRangePop() { return 0; }

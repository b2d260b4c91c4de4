// A host-only stand-in for the HIP runtime calls and kernel launchers the
// library's host code makes (test infrastructure only), so that host.cpp's
// bookkeeping (batches, captured graphs and their caches, job and segment
// tables, stream forks and joins) runs on a CPU under AddressSanitizer and
// UndefinedBehaviorSanitizer.  "Device" memory is host memory; copies and
// fills act on it; kernels do nothing except that every launch checks that
// the memory it would touch is live, and a captured graph keeps those
// pointers so that a later launch of the graph checks them again (a graph
// that outlives its tables or batch state aborts here).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include "../../paper_2601_18140_amd/csrc/internal.h"
#include "../../paper_2601_18140_amd/csrc/levelize.h"

namespace {

std::mutex mu;
std::map<const char*, size_t> live;  // allocation start -> bytes
std::set<const void*> streams, events, graphs, execs;
std::map<const void*, std::vector<const void*>> capturing;  // stream -> pointers launched
std::map<const void*, const void*> joined;   // stream forked into a capture -> capturing stream
std::map<const void*, const void*> marks;    // event recorded in a capture -> capturing stream
std::map<const void*, std::vector<const void*>> graph_ptrs, exec_ptrs;
alignas(256) uint64_t scratch_mock[1 << 20];

[[noreturn]] void die(const char* what, const void* p) {
  std::fprintf(stderr, "hip_mock: %s (%p)\n", what, p);
  std::abort();
}

// p (non-null) must lie inside a live allocation, or the mock scratch.
void check_ptr(const void* p) {
  if (!p) return;
  const char* c = (const char*)p;
  if (c >= (const char*)scratch_mock && c < (const char*)scratch_mock + sizeof scratch_mock) return;
  auto it = live.upper_bound(c);
  if (it == live.begin()) die("pointer outside every allocation", p);
  --it;
  if (c >= it->first + std::max<size_t>(it->second, 1)) die("pointer outside every allocation", p);
}

// A kernel launch on stream s touching pointers ps: checked now, and kept
// when s is being captured.
void launched(hipStream_t s, std::initializer_list<const void*> ps) {
  std::lock_guard<std::mutex> lk(mu);
  if (s && !streams.count(s)) die("launch on an unknown stream", s);
  for (const void* p : ps) check_ptr(p);
  auto j = joined.find(s);
  auto it = capturing.find(j != joined.end() ? j->second : (const void*)s);
  if (it != capturing.end()) it->second.insert(it->second.end(), ps.begin(), ps.end());
}

}  // namespace

extern "C" {

hipError_t hipMalloc(void** p, size_t n) {
  std::lock_guard<std::mutex> lk(mu);
  char* q = (char*)std::aligned_alloc(256, (n + 255) & ~size_t(255));
  if (!q) return hipErrorOutOfMemory;
  std::memset(q, 0xA5, (n + 255) & ~size_t(255));
  live[q] = n;
  *p = q;
  return hipSuccess;
}

hipError_t hipFree(void* p) {
  std::lock_guard<std::mutex> lk(mu);
  if (!p) return hipSuccess;
  auto it = live.find((const char*)p);
  if (it == live.end()) die("hipFree of an unknown pointer", p);
  live.erase(it);
  std::free(p);
  return hipSuccess;
}

static void copy_check(const void* p, size_t n) {
  std::lock_guard<std::mutex> lk(mu);
  const char* c = (const char*)p;
  auto it = live.upper_bound(c);
  if (it == live.begin()) return;  // host memory
  --it;
  if (c >= it->first + it->second) return;  // host memory
  if (c + n > it->first + it->second) die("copy past the end of a device allocation", p);
}

hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  copy_check(d, n);
  copy_check(s, n);
  std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k) {
  return hipMemcpyAsync(d, s, n, k, nullptr);
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  copy_check(d, n);
  std::memset(d, v, n);
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  std::lock_guard<std::mutex> lk(mu);
  *s = (hipStream_t)new char[1];
  streams.insert(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::mutex> lk(mu);
  if (!streams.erase(s)) die("hipStreamDestroy of an unknown stream", s);
  delete[] (char*)s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  std::lock_guard<std::mutex> lk(mu);
  if (s && !streams.count(s)) die("sync of an unknown stream", s);
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
  std::lock_guard<std::mutex> lk(mu);
  *e = (hipEvent_t)new char[1];
  events.insert(*e);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(mu);
  if (!events.erase(e)) die("hipEventDestroy of an unknown event", e);
  delete[] (char*)e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::lock_guard<std::mutex> lk(mu);
  if (!events.count(e)) die("record of an unknown event", e);
  if (s && !streams.count(s)) die("record on an unknown stream", s);
  auto j = joined.find(s);
  const void* root = j != joined.end() ? j->second : (const void*)s;
  if (capturing.count(root)) marks[e] = root;
  else marks.erase(e);
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 1.0f;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  std::lock_guard<std::mutex> lk(mu);
  if (!events.count(e)) die("wait for an unknown event", e);
  if (s && !streams.count(s)) die("wait on an unknown stream", s);
  // A stream that waits for an event recorded on a capturing stream joins
  // the capture (fork); its launches belong to the same graph.
  auto m = marks.find(e);
  if (m != marks.end() && m->second != (const void*)s) joined[s] = m->second;
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  std::lock_guard<std::mutex> lk(mu);
  if (capturing.count(s)) die("capture begun twice", s);
  capturing[s] = {};
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  std::lock_guard<std::mutex> lk(mu);
  auto it = capturing.find(s);
  if (it == capturing.end()) die("capture ended but not begun", s);
  *g = (hipGraph_t)new char[1];
  graphs.insert(*g);
  graph_ptrs[*g] = it->second;
  capturing.erase(it);
  for (auto q = joined.begin(); q != joined.end();)
    q = q->second == (const void*)s ? joined.erase(q) : std::next(q);
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  std::lock_guard<std::mutex> lk(mu);
  if (!graphs.count(g)) die("instantiate of an unknown graph", g);
  *x = (hipGraphExec_t)new char[1];
  execs.insert(*x);
  exec_ptrs[*x] = graph_ptrs[g];
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  std::lock_guard<std::mutex> lk(mu);
  if (!graphs.erase(g)) die("destroy of an unknown graph", g);
  graph_ptrs.erase(g);
  delete[] (char*)g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  std::lock_guard<std::mutex> lk(mu);
  if (!execs.erase(x)) die("destroy of an unknown graph exec", x);
  exec_ptrs.erase(x);
  delete[] (char*)x;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  std::lock_guard<std::mutex> lk(mu);
  if (!execs.count(x)) die("launch of a destroyed or unknown graph exec", x);
  if (s && !streams.count(s)) die("graph launch on an unknown stream", s);
  for (const void* p : exec_ptrs[x]) check_ptr(p);
  return hipSuccess;
}
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
  std::memset(p, 0, sizeof *p);
  std::strcpy(p->gcnArchName, "gfx950-mock");
  p->multiProcessorCount = 256;
  p->maxSharedMemoryPerMultiProcessor = 160 * 1024;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void*) {
  *p = scratch_mock;
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock error"; }
void** __hipRegisterFatBinary(const void*) {
  static void* h = nullptr;
  return &h;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterVar(void**, void*, char*, const char*, int, size_t, int, int) {}

}  // extern "C"

// Kernel launchers: nothing runs; the memory they would touch must be live.
namespace rteaal {

hipError_t launch_resident(const ResJob& J, uint32_t, uint32_t, uint32_t, bool, bool, uint32_t,
                           hipStream_t s) {
  launched(s, {J.ops, J.layers, J.state, J.seeds, J.ctl, J.regs, J.digest});
  return hipSuccess;
}
hipError_t launch_resident_multi(const ResJob* jobs, const uint2* map, uint32_t, uint32_t, bool,
                                 bool, uint32_t, size_t, hipStream_t s) {
  launched(s, {jobs, map});
  return hipSuccess;
}
size_t resident_lds_bytes(const StateLayout& L, uint32_t n_ops_total, uint32_t n_layers,
                          bool lds_state, bool lds_ops) {
  size_t b = lds_state ? L.pitch : 0;
  if (lds_ops) b += (size_t)n_ops_total * sizeof(DevOp) + (size_t)n_layers * sizeof(DevLayer);
  return b;
}
size_t resident_max_lds() { return 160u * 1024u - 256u; }
hipError_t launch_sweep_light(const Program& p, const StateLayout&, char* state, const OpRanges&,
                              uint32_t, uint32_t, uint32_t, uint32_t, TilePass, hipStream_t s) {
  launched(s, {p.ops, state});
  return hipSuccess;
}
hipError_t launch_sweep_heavy(const Program& p, const StateLayout&, char* state,
                              const uint64_t* seeds, const DevCtl* ctl, uint32_t, uint32_t,
                              const DevLayer&, uint32_t, uint32_t, TilePass, hipStream_t s) {
  launched(s, {p.ops, p.layers, state, seeds, ctl});
  return hipSuccess;
}
hipError_t launch_layer(const ResJob& J, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t,
                        hipStream_t s) {
  launched(s, {J.ops, J.layers, J.state, J.seeds, J.ctl});
  return hipSuccess;
}
hipError_t launch_layer_persistent(const ResJob& J, uint32_t, uint32_t, GridSync* gs, uint64_t* acc,
                                   uint32_t, uint32_t, hipStream_t s) {
  launched(s, {J.ops, J.state, gs, acc, J.digest, J.regs});
  std::memset(gs, 0, sizeof *gs);  // the real launch clears the barrier state first
  return hipSuccess;
}
uint32_t partitioned_capacity(uint32_t, bool, size_t) { return 256u * 8u; }
hipError_t launch_partitioned(const PartRun& R, uint32_t, bool, hipStream_t s) {
  launched(s, {R.parts, R.const_limbs, R.regs, R.state, R.seeds, R.ctl, R.xch, R.acc, R.digest,
               R.gs});
  copy_check(R.acc, (size_t)R.n_inst * 3 * 8);
  copy_check(R.state, (size_t)R.n_inst * R.n_parts * R.pitch);
  copy_check(R.xch, (size_t)R.n_inst * 2 * R.reg_words * 8);
  for (uint32_t p = 0; p < R.n_parts; ++p) {  // the job table's pointers must be live too
    const PartJob& J = R.parts[p];
    launched(s, {J.ops, J.layers, J.own, J.need});
    copy_check(J.layers, (size_t)J.n_layers * sizeof(DevLayer));
    if (J.n_own) copy_check(J.own, (size_t)J.n_own * 4);
    if (J.n_need) copy_check(J.need, (size_t)J.n_need * 4);
  }
  std::memset(R.gs, 0, sizeof *R.gs);
  return hipSuccess;
}
hipError_t launch_advance(DevCtl* ctl, uint64_t, hipStream_t s) {
  launched(s, {ctl});
  return hipSuccess;
}
hipError_t launch_set_words(DevCtl* ctl, const uint64_t* words, hipStream_t s) {
  launched(s, {ctl, words});
  return hipSuccess;
}
hipError_t launch_pack(bool, const StateLayout&, const char* state, const SlotRef* refs, uint32_t,
                       uint32_t wpi, uint32_t, uint32_t n, uint64_t* out, hipStream_t s) {
  launched(s, {state, refs, out});
  copy_check(out, (size_t)wpi * n * 8);
  std::memset(out, 0, (size_t)wpi * n * 8);
  return hipSuccess;
}
hipError_t launch_unpack(bool, const StateLayout&, char* state, const SlotRef* refs, uint32_t,
                         uint32_t, uint32_t, uint32_t, const uint64_t* in, hipStream_t s) {
  launched(s, {state, refs, in});
  return hipSuccess;
}
hipError_t launch_capture(bool, const StateLayout&, const char* state, const SlotRef* refs, uint32_t,
                          uint64_t* shadow, uint32_t, bool, const DevCtl* ctl, ChangeRec* log,
                          uint64_t, unsigned long long* count, hipStream_t s) {
  launched(s, {state, refs, shadow, ctl, log, count});
  return hipSuccess;
}
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s) {
  launched(s, {p});
  copy_check(p, n * 8);
  for (uint64_t i = 0; i < n; ++i) p[i] = v;
  return hipSuccess;
}
hipError_t launch_digest(bool, const StateLayout&, const char* state, const SlotRef* regs, uint32_t,
                         uint32_t, uint64_t* digest, uint64_t* acc, hipStream_t s) {
  launched(s, {state, regs, digest, acc});
  return hipSuccess;
}
void digest_shape(bool sweep, uint32_t n_regs, uint32_t n_inst, uint32_t* n_units, uint32_t* per) {
  *n_units = sweep ? (n_inst + 63u) / 64u : n_inst;
  const uint64_t want = std::max<uint64_t>(1, (16384u + *n_units - 1) / *n_units);
  uint64_t q = ((uint64_t)std::max<uint32_t>(n_regs, 1u) + want - 1) / want;
  if (sweep) q = std::max<uint64_t>(q, 32u);
  else q = (q + 63u) & ~uint64_t(63);
  *per = (uint32_t)q;
}
bool multi_mixable(uint32_t kind, uint32_t tg) {
  return kind == 3 || ((kind == 0 || kind == 2) && tg <= 4) || (kind == 1 && tg <= 2);
}
bool multi_lean(uint32_t kind, uint32_t tg, bool narrow) {
  return (kind == 0 && tg <= 2) || (kind == 1 && (tg == 1 || (narrow && tg == 2))) || kind == 3;
}
uint32_t multi_variant(uint32_t kind, uint32_t tg, uint32_t unroll, bool lean, bool narrow) {
  const uint32_t lg = tg >= 4 ? 2u : tg >= 2 ? 1u : 0u;
  uint32_t lu = 0;
  if (kind == 0) {
    if (unroll == 2 && tg <= 4) lu = 1;
    if (unroll == 4 && tg <= 2) lu = 2;
    if (lean && lu == 1 && tg > 2) lu = 0;
    if (lean && lu == 2 && tg > 1) lu = 1;  // the lean kernel runs 4 in flight on one tile only
  }
  return kind * 8u + lg + 64u * lu + (kind == 1 && narrow ? 256u : 0u);
}
hipError_t launch_multi(uint32_t kind, uint32_t, const MultiSeg* segs, const uint32_t* wave0,
                        uint32_t n_seg, uint64_t n_waves, hipStream_t s) {
  launched(s, {segs, wave0, segs + n_seg - 1, wave0 + n_seg});
  if (wave0[n_seg] != n_waves) die("segment prefix does not match the wave count", wave0);
  copy_check(wave0, (n_seg + 1 + n_waves) * 4);  // the per-wavefront segment table follows
  for (uint64_t w = 0; w < n_waves; ++w) {
    const uint32_t k = wave0[n_seg + 1 + w];
    if (k >= n_seg || w < wave0[k] || w >= wave0[k + 1]) die("wavefront segment table", &wave0[n_seg + 1 + w]);
  }
  for (uint32_t k = 0; k < n_seg; ++k) {
    const uint32_t vk = (segs[k].variant % 64) / 8, vt = 1u << (segs[k].variant % 8);
    const uint32_t vu = 1u << ((segs[k].variant % 256) / 64);
    const bool vn = segs[k].variant >= 256;
    if (vn && vk != 1) die("two-limb variant on a piece that is not heavy", &segs[k]);
    if ((kind == 4 || kind == 5) && vu > 1 && (vk != 0 || vu > 4 || (vu == 4 && vt > 2) || vt > 4))
      die("mixed segment with an unroll depth outside the kernel's variants", &segs[k]);
    if (kind == 4 && !multi_mixable(vk, vt)) die("mixed segment of an unknown variant", &segs[k]);
    if ((kind == 5 || kind == 6) && (!multi_lean(vk, vt, vn) || (vu == 2 && vt > 2) || (vu == 4 && vt > 1)))
      die("lean mixed segment of a variant outside the lean set", &segs[k]);
    if (kind == 6 && (vk == 3 || vu > 2 || (vk == 1 && vt > 1)))
      die("smallest mixed set with a LAYERED piece or 4 in flight", &segs[k]);
    launched(s, {segs[k].ops, segs[k].layers, segs[k].const_limbs, segs[k].state, segs[k].seeds,
                 segs[k].ctl});
    if (wave0[k + 1] <= wave0[k]) die("empty or decreasing segment", &wave0[k]);
  }
  return hipSuccess;
}
hipError_t launch_digest_multi(const DigestSeg* segs, const uint32_t* wave0, uint32_t n_seg,
                               uint64_t n_waves, uint32_t, hipStream_t s) {
  launched(s, {segs, wave0, segs + n_seg - 1, wave0 + n_seg});
  if (wave0[n_seg] != n_waves) die("digest prefix does not match the wave count", wave0);
  for (uint32_t k = 0; k < n_seg; ++k)
    launched(s, {segs[k].state, segs[k].regs, segs[k].digest, segs[k].acc, segs[k].ctl});
  return hipSuccess;
}
hipError_t levelize_temp_bytes(uint32_t, size_t* bytes) {
  *bytes = 256;
  return hipSuccess;
}
hipError_t levelize_run(const LvBuffers&, uint32_t, uint32_t, uint32_t, hipStream_t, LvResult*) {
  return hipErrorNotSupported;
}

}  // namespace rteaal

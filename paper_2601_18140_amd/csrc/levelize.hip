// Device levelizer for gfx950: layers of a dataflow graph given in any
// operation order (paper section "Evaluating Arbitrary Dataflow Graphs"; the
// compiler slices the graph into layers by topological sort).
//
// A frontier sweep over the graph (Kahn's order, one launch per layer):
//   1. producer[slot] = the operation writing it (a second writer is an
//      error);
//   2. in-degree of every operation = its operand entries fed by an
//      operation; out-degree of the producers;
//   3. consumer lists (CSR) from an exclusive scan of the out-degrees;
//   4. layer 0 = operations with in-degree 0; each step labels the frontier
//      with the layer and decrements its consumers, whose last decrement
//      puts them in the next frontier.  An operation thus lands in the layer
//      1 + max(layers of its producers).  Operations never reached lie on or
//      behind a cycle.  Frontier appends are counted once per block (all
//      blocks share one counter, whose atomics serialize), and the steps run
//      in chunks of launches with one read-back per chunk;
//   5. a stable radix sort of (layer, index) gives the order, and the first
//      position of every layer value gives the layer ranges.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>

#include "levelize.h"

namespace rteaal {
namespace {

constexpr uint32_t kBlock = 256;

uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

__global__ void k_lv_fill(uint32_t* p, uint32_t v, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_lv_iota(uint32_t* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

__global__ void k_lv_producer(const uint32_t* __restrict__ dst, uint32_t n, uint32_t* producer,
                              uint32_t* dup_slot) {
  const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const uint32_t d = dst[o];
  if (atomicCAS(&producer[d], kLvNone, o) != kLvNone) atomicMin(dup_slot, d);
}

__global__ void k_lv_degrees(const uint32_t* __restrict__ src_ptr, const uint32_t* __restrict__ src,
                             const uint32_t* __restrict__ producer, uint32_t n, uint32_t* indeg,
                             uint32_t* outdeg) {
  const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  uint32_t cnt = 0;
  for (uint32_t e = src_ptr[o]; e < src_ptr[o + 1]; ++e) {
    const uint32_t p = producer[src[e]];
    if (p != kLvNone) {
      ++cnt;
      atomicAdd(&outdeg[p], 1u);
    }
  }
  indeg[o] = cnt;
}

__global__ void k_lv_consumers(const uint32_t* __restrict__ src_ptr, const uint32_t* __restrict__ src,
                               const uint32_t* __restrict__ producer, uint32_t n,
                               const uint32_t* __restrict__ out_ptr, uint32_t* cursor,
                               uint32_t* out_idx) {
  const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  for (uint32_t e = src_ptr[o]; e < src_ptr[o + 1]; ++e) {
    const uint32_t p = producer[src[e]];
    if (p != kLvNone) out_idx[out_ptr[p] + atomicAdd(&cursor[p], 1u)] = o;
  }
}

constexpr uint32_t kBig = 1024;  // threads per block of the frontier kernels

// Appends `item` to list when `take`, with one atomic on the shared count per
// block: the block's takers get consecutive places.  Every thread of the
// block calls it; s is two words of LDS.
__device__ __forceinline__ void block_append(bool take, uint32_t item, uint32_t* list,
                                             uint32_t* count, uint32_t* s) {
  const uint32_t lane = threadIdx.x & 63u;
  if (threadIdx.x == 0) s[0] = 0;
  __syncthreads();
  const uint64_t m = __ballot(take);
  const uint32_t leader = m ? (uint32_t)__ffsll((unsigned long long)m) - 1u : 0u;
  uint32_t wbase = 0;
  if (m && lane == leader) wbase = atomicAdd(&s[0], (uint32_t)__popcll(m));
  wbase = __shfl(wbase, (int)leader);
  __syncthreads();
  if (threadIdx.x == 0) s[1] = s[0] ? atomicAdd(count, s[0]) : 0u;
  __syncthreads();
  if (take) list[s[1] + wbase + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = item;
  __syncthreads();
}

__global__ void __launch_bounds__(kBig) k_lv_roots(const uint32_t* __restrict__ indeg, uint32_t n,
                                                   uint32_t* front, uint32_t* count) {
  __shared__ uint32_t s[2];
  const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
  block_append(o < n && indeg[o] == 0, o, front, count, s);
}

// One layer L of the sweep: labels the frontier (its size in *count_in, as
// the previous step left it) with L and collects the operations whose last
// producer it holds into front_out / *count_out.  Records the frontier size
// in sizes[L] and clears the counter the next step appends to.  The grid
// strides over the frontier; the threads of a block walk their consumer
// lists in step, so every step of the walk is one block-wide append.
__global__ void __launch_bounds__(kBig)
k_lv_step(const uint32_t* __restrict__ front_in, const uint32_t* count_in, uint32_t L,
          const uint32_t* __restrict__ out_ptr, const uint32_t* __restrict__ out_idx,
          uint32_t* indeg, uint32_t* layer, uint32_t* front_out, uint32_t* count_out,
          uint32_t* count_next, uint32_t* sizes) {
  __shared__ uint32_t s[2];
  const uint32_t n_in = *count_in;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sizes[L] = n_in;
    *count_next = 0;
  }
  for (uint32_t base = blockIdx.x * blockDim.x; base < n_in; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t e = 0, e1 = 0;
    if (i < n_in) {
      const uint32_t o = front_in[i];
      layer[o] = L;
      e = out_ptr[o];
      e1 = out_ptr[o + 1];
    }
    while (__syncthreads_or(e < e1)) {
      bool ready = false;
      uint32_t c = 0;
      if (e < e1) {
        c = out_idx[e];
        ready = atomicSub(&indeg[c], 1u) == 1u;
        ++e;
      }
      block_append(ready, c, front_out, count_out, s);
    }
  }
}

// Range checks of the graph on the device, before any kernel indexes with
// it: bad[0] = first operation whose operand range decreases, bad[1] = first
// operand entry naming a slot >= n_slots, bad[2] = first operation writing
// one (kLvNone when none).
__global__ void k_lv_check(const uint32_t* __restrict__ src_ptr, const uint32_t* __restrict__ src,
                           const uint32_t* __restrict__ dst, uint32_t n, uint32_t ne,
                           uint32_t n_slots, uint32_t* bad) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (src_ptr[i + 1] < src_ptr[i]) atomicMin(&bad[0], i);
    if (dst[i] >= n_slots) atomicMin(&bad[2], i);
  }
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < ne; k += stride)
    if (src[k] >= n_slots) atomicMin(&bad[1], k);
}

// Every layer value 0 .. n_layers-1 occurs (an operation of layer k > 0 has a
// producer in layer k - 1), so each one's first position is written.
__global__ void k_lv_bounds(const uint32_t* __restrict__ keys, uint32_t n, uint32_t* layer_ptr) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (i == 0 || keys[i] != keys[i - 1])) layer_ptr[keys[i]] = i;
}

uint32_t bits_for(uint32_t v) {
  uint32_t b = 1;
  while (b < 32 && (v >> b) != 0) ++b;
  return b;
}

}  // namespace

hipError_t levelize_temp_bytes(uint32_t n, size_t* bytes) {
  size_t a = 0, b = 0;
  hipError_t e = rocprim::exclusive_scan(nullptr, a, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                         0u, (size_t)n + 1, rocprim::plus<uint32_t>());
  if (e != hipSuccess) return e;
  e = rocprim::radix_sort_pairs(nullptr, b, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                (const uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)n, 0u, 32u);
  *bytes = std::max(a, b);
  return e;
}

hipError_t levelize_run(const LvBuffers& B, uint32_t n_slots, uint32_t n, uint32_t ne,
                        hipStream_t s, LvResult* out) {
  hipError_t e;
#define LV_TRY(expr)              \
  do {                            \
    e = (expr);                   \
    if (e != hipSuccess) return e; \
  } while (0)
  out->n_layers = 0;
  out->processed = 0;
  out->dup_slot = kLvNone;
  out->bad[0] = out->bad[1] = out->bad[2] = kLvNone;
  uint32_t* dup = B.scalars;          // smallest slot with two writers
  uint32_t* cnt = B.scalars + 1;      // three rotating frontier counters
  uint32_t* bad = B.scalars + 4;      // range-check results
  // 0. range checks, before any kernel indexes with the graph.
  hipLaunchKernelGGL(k_lv_fill, dim3(1), dim3(kBlock), 0, s, B.scalars, kLvNone, (uint64_t)8);
  const uint32_t gcheck = std::min<uint32_t>(blocks_for(std::max(n, ne)), 4096u);
  hipLaunchKernelGGL(k_lv_check, dim3(gcheck), dim3(kBlock), 0, s, B.src_ptr, B.src, B.dst, n, ne,
                     n_slots, bad);
  LV_TRY(hipGetLastError());
  uint32_t host_bad[3];
  LV_TRY(hipMemcpyAsync(host_bad, bad, sizeof host_bad, hipMemcpyDeviceToHost, s));
  LV_TRY(hipStreamSynchronize(s));
  if (host_bad[0] != kLvNone || host_bad[1] != kLvNone || host_bad[2] != kLvNone) {
    for (int k = 0; k < 3; ++k) out->bad[k] = host_bad[k];
    return hipSuccess;
  }
  // 1. producers.
  hipLaunchKernelGGL(k_lv_fill, dim3(blocks_for(n_slots)), dim3(kBlock), 0, s, B.producer, kLvNone,
                     (uint64_t)n_slots);
  hipLaunchKernelGGL(k_lv_producer, dim3(blocks_for(n)), dim3(kBlock), 0, s, B.dst, n, B.producer,
                     dup);
  LV_TRY(hipGetLastError());
  uint32_t host_dup = kLvNone;
  LV_TRY(hipMemcpyAsync(&host_dup, dup, 4, hipMemcpyDeviceToHost, s));
  LV_TRY(hipStreamSynchronize(s));
  if (host_dup != kLvNone) {
    out->dup_slot = host_dup;
    return hipSuccess;
  }
  // 2. degrees.
  hipLaunchKernelGGL(k_lv_fill, dim3(blocks_for(n + 1ull)), dim3(kBlock), 0, s, B.outdeg, 0u,
                     (uint64_t)n + 1);
  hipLaunchKernelGGL(k_lv_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, B.cursor, 0u, (uint64_t)n);
  hipLaunchKernelGGL(k_lv_degrees, dim3(blocks_for(n)), dim3(kBlock), 0, s, B.src_ptr, B.src,
                     B.producer, n, B.indeg, B.outdeg);
  LV_TRY(hipGetLastError());
  // 3. consumer lists.
  size_t tb = B.temp_bytes;
  LV_TRY(rocprim::exclusive_scan(B.temp, tb, B.outdeg, B.out_ptr, 0u, (size_t)n + 1,
                                 rocprim::plus<uint32_t>(), s));
  hipLaunchKernelGGL(k_lv_consumers, dim3(blocks_for(n)), dim3(kBlock), 0, s, B.src_ptr, B.src,
                     B.producer, n, B.out_ptr, B.cursor, B.out_idx);
  LV_TRY(hipGetLastError());
  // 4. frontier sweep.  Layer L reads counter L % 3, appends to (L+1) % 3 and
  // clears (L+2) % 3; the roots go to counter 0.  Steps are launched in
  // chunks without waiting; after each chunk the recorded frontier sizes tell
  // whether the sweep has ended (a step over an empty frontier does nothing).
  hipLaunchKernelGGL(k_lv_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, B.layer, kLvNone, (uint64_t)n);
  hipLaunchKernelGGL(k_lv_fill, dim3(1), dim3(kBlock), 0, s, cnt, 0u, (uint64_t)3);
  hipLaunchKernelGGL(k_lv_roots, dim3((n + kBig - 1) / kBig), dim3(kBig), 0, s, B.indeg, n,
                     B.front[0], cnt);
  LV_TRY(hipGetLastError());
  const uint32_t gstep = std::min<uint32_t>((n + kBig - 1) / kBig, 2048u);
  constexpr uint32_t kChunk = 8;
  uint32_t L = 0, done = 0;
  for (bool more = true; more;) {
    for (uint32_t j = 0; j < kChunk; ++j, ++L)
      hipLaunchKernelGGL(k_lv_step, dim3(gstep), dim3(kBig), 0, s, B.front[L & 1], cnt + L % 3, L,
                         B.out_ptr, B.out_idx, B.indeg, B.layer, B.front[(L + 1) & 1],
                         cnt + (L + 1) % 3, cnt + (L + 2) % 3, B.sizes);
    LV_TRY(hipGetLastError());
    uint32_t sz[kChunk];
    LV_TRY(hipMemcpyAsync(sz, B.sizes + (L - kChunk), sizeof sz, hipMemcpyDeviceToHost, s));
    LV_TRY(hipStreamSynchronize(s));
    for (uint32_t j = 0; j < kChunk && more; ++j) {
      if (sz[j] == 0) {
        more = false;
        L = L - kChunk + j;  // layers 0 .. L-1 are non-empty
      } else {
        done += sz[j];
      }
    }
  }
  out->n_layers = L;
  out->processed = done;
  if (done < n) return hipSuccess;
  // 5. order and layer ranges.
  hipLaunchKernelGGL(k_lv_iota, dim3(blocks_for(n)), dim3(kBlock), 0, s, B.vals_in, n);
  tb = B.temp_bytes;
  LV_TRY(rocprim::radix_sort_pairs(B.temp, tb, B.layer, B.keys_out, B.vals_in, B.order, (size_t)n,
                                   0u, bits_for(L - 1), s));
  hipLaunchKernelGGL(k_lv_bounds, dim3(blocks_for(n)), dim3(kBlock), 0, s, B.keys_out, n,
                     B.layer_ptr);
  hipLaunchKernelGGL(k_lv_fill, dim3(1), dim3(kBlock), 0, s, B.layer_ptr + L, n, (uint64_t)1);
  LV_TRY(hipGetLastError());
#undef LV_TRY
  return hipSuccess;
}

}  // namespace rteaal

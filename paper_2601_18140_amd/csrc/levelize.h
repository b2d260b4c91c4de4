// Internal interface of the device levelizer (levelize.hip), used by the
// host runtime's rteaal_levelize.  Not part of the public C interface.
//
// Levelization (paper section "Evaluating Arbitrary Dataflow Graphs", and
// the compiler's slicing of the dataflow graph by topological sort): every
// operation gets layer 1 + the largest layer among the producers of its
// operands, 0 when all its operands are sources (slots no operation writes).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rteaal {

constexpr uint32_t kLvNone = 0xffffffffu;

// Device buffers of one levelization (n operations, e operand entries,
// n_slots slots).  The caller allocates them with the sizes below and
// uploads src_ptr [n + 1], src [e] and dst [n].
struct LvBuffers {
  const uint32_t* src_ptr;
  const uint32_t* src;
  const uint32_t* dst;
  uint32_t* producer;  // [n_slots]   operation writing each slot, or kLvNone
  uint32_t* indeg;     // [n]         operand entries fed by an operation
  uint32_t* outdeg;    // [n + 1]     consumers of each operation (last entry 0)
  uint32_t* out_ptr;   // [n + 1]     consumer ranges (exclusive scan of outdeg)
  uint32_t* cursor;    // [n]         fill cursors of the consumer lists
  uint32_t* out_idx;   // [e]         consumers of each operation
  uint32_t* front[2];  // [n] each    current and next frontier
  uint32_t* layer;     // [n]         result: layer of each operation
  uint32_t* keys_out;  // [n]         layers sorted
  uint32_t* vals_in;   // [n]         0 .. n-1
  uint32_t* order;     // [n]         result: operations sorted by (layer, index)
  uint32_t* layer_ptr; // [n + 1]     result: layer ranges in `order`
  uint32_t* sizes;     // [n + 16]    frontier size of every layer step
  uint32_t* scalars;   // [8]         duplicate-writer slot, frontier counters, range checks
  void* temp;          // scan / sort scratch of levelize_temp_bytes(n) bytes
  size_t temp_bytes;
};

// Scratch bytes the scan and the sort of n operations need.
hipError_t levelize_temp_bytes(uint32_t n, size_t* bytes);

// Outcome of a levelization.
struct LvResult {
  uint32_t n_layers;   // layers assigned
  uint32_t processed;  // operations that received a layer (< n: a cycle)
  uint32_t dup_slot;   // a slot written by two operations, or kLvNone
  uint32_t bad[3];     // first decreasing operand range (operation), first
                       // operand entry and first operation naming a slot
                       // >= n_slots; kLvNone when the graph is in range
};

// Runs the levelization of n >= 1 operations with ne operand entries on
// stream s (src_ptr[0] = 0 and src_ptr[n] = ne are the caller's to check).
// Returns when the device work is done.  Stops early when the graph is out
// of range (bad set) or a slot has two writers (dup_slot set).  When
// processed < n, `layer` holds kLvNone for the operations on or behind a
// cycle and the order is not computed.
hipError_t levelize_run(const LvBuffers& B, uint32_t n_slots, uint32_t n, uint32_t ne,
                        hipStream_t s, LvResult* out);

}  // namespace rteaal

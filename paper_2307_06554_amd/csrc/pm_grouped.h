// Persistent grouped kernel: products of uneven degree and modulus in one launch.
//
// Work items come from a device table sorted by decreasing cost (largest first)
// and are claimed with one atomic add per item (a dynamic list schedule, which
// with that order approximates longest-processing-time-first).  Resident groups
// run with as many int8 limbs as their modulus needs.  Each item is a
// group of four 32x32 tiles of LDS-resident products (degrees 4..4096), a group
// of products on 16x16 tiles (64..512, where the tile table says so) or one
// 64x64 block of a K-streamed product (every other degree).  Algorithm 1's
// GenConfig / ExtractDimensions run once on the host when the plan is built;
// the launch only reads the resulting job table.
#pragma once
#include "pm_mfma32.h"
#include "pm_mfma16.h"
#include "pm_stream.h"

namespace pm {

enum : uint32_t { kJobResident = 0, kJobStream = 1, kJobSmall = 2 };

struct GroupJob {
  uint32_t kind;
  uint32_t L;        // int8 limbs of a resident group: 2, 3 or 4 (from its modulus)
  uint32_t pad[2];
  Mfma32Params rp;   // kind == kJobResident, or kJobSmall (16x16 tiles, rp.slots products per item)
  StreamParams sp;   // kind == kJobStream (4 limbs)
};

struct WorkItem {
  uint32_t group;    // index into the GroupJob table
  uint32_t index;    // resident: tile-group index; small: group of rp.slots products;
                     // stream: product * ublocks + u-block
};

template <int L>
__device__ __forceinline__ void resident_item(const Mfma32Params& P, uint32_t index, uint8_t* smem) {
  if (P.kparts > 1) resident_group_split<L>(P, index, smem);
  else resident_group<L, false>(P, index, smem);
}
template <int L>
__device__ __forceinline__ void small_item(const Mfma32Params& P, uint32_t index, uint8_t* smem) {
  small_group<L>(P, index, smem, (Slot16*)(smem + P.slots * P.slot_bytes));
}

// The first grid items (largest first) are dealt out statically: workgroup b < G/2
// takes item b and workgroup G/2 + k item G - 1 - k (G = grid, no larger than the
// list), so that the workgroups the dispatcher places on one CU first, b and b + G/2,
// pair a larger item with a smaller one; every later item comes from the queue,
// whose k-th claim is item G + k.  A workgroup claims its next item when its current
// one is done, so that the queue hands the remaining items (the smallest) to the
// workgroups that come free first; a list no longer than the grid needs no queue.
// counter[0] is the queue, counter[1] counts the workgroups that have left; the last
// to leave sets both back to zero, so that the next launch (a graph replay) starts
// from an empty queue without a reset node.  Every workgroup's final claim has
// returned before it counts itself out, so no claim can follow the reset.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void grouped_kernel(const GroupJob* __restrict__ jobs, const WorkItem* __restrict__ items, uint32_t nitems,
                    uint32_t* counter) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint32_t next_item;
  const uint32_t half = gridDim.x >> 1;
  uint32_t it = blockIdx.x < half ? blockIdx.x : gridDim.x - 1 - (blockIdx.x - half);
  const bool queue = nitems > gridDim.x;
  for (;;) {
    const WorkItem w = items[it];
    const GroupJob& job = jobs[w.group];
    if (job.kind == kJobResident) {
      switch (job.L) {
        case 2: resident_item<2>(job.rp, w.index, smem); break;
        case 3: resident_item<3>(job.rp, w.index, smem); break;
        default: resident_item<4>(job.rp, w.index, smem); break;
      }
    } else if (job.kind == kJobSmall) {
      switch (job.L) {
        case 2: small_item<2>(job.rp, w.index, smem); break;
        case 3: small_item<3>(job.rp, w.index, smem); break;
        default: small_item<4>(job.rp, w.index, smem); break;
      }
    } else {
      stream_block<4, uint32_t>(job.sp, w.index, smem);
    }
    if (!queue) break;  // every item was dealt out: no claims, nothing to reset
    if (threadIdx.x == 0) next_item = atomicAdd(counter, 1u) + gridDim.x;
    __syncthreads();  // LDS is reused by the next item; next_item is visible
    it = next_item;
    if (it >= nitems) {  // uniform: every wave leaves together
      if (threadIdx.x == 0 && atomicAdd(counter + 1, 1u) == gridDim.x - 1) {
        atomicExch(counter, 0u);
        atomicExch(counter + 1, 0u);
      }
      break;
    }
    __syncthreads();  // every wave has read next_item before it is written again
  }
}

}  // namespace pm

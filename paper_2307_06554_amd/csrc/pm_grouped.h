// Persistent grouped kernel: products of uneven degree and modulus in one launch.
//
// Work items come from a device table sorted by decreasing cost (largest first)
// and are claimed with one atomic add per item (a dynamic list schedule, which
// with that order approximates longest-processing-time-first).  Each item is a
// group of four 32x32 tiles of LDS-resident products (degrees 4..4096) or one
// 64x64 block of a K-streamed product (every other degree).  Algorithm 1's
// GenConfig / ExtractDimensions run once on the host when the plan is built;
// the launch only reads the resulting job table.
#pragma once
#include "pm_mfma32.h"
#include "pm_stream.h"

namespace pm {

enum : uint32_t { kJobResident = 0, kJobStream = 1 };

struct GroupJob {
  uint32_t kind;
  uint32_t pad[3];
  Mfma32Params rp;   // kind == kJobResident
  StreamParams sp;   // kind == kJobStream
};

struct WorkItem {
  uint32_t group;    // index into the GroupJob table
  uint32_t index;    // resident: tile-group index; stream: product * ublocks + u-block
};

// counter[0] is the queue, counter[1] counts the workgroups that have left; the last
// to leave sets both back to zero, so that the next launch (a graph replay) starts
// from an empty queue without a reset node.  Every workgroup's final claim has
// returned before it counts itself out, so no claim can follow the reset.
template <int L>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void grouped_kernel(const GroupJob* __restrict__ jobs, const WorkItem* __restrict__ items, uint32_t nitems,
                    uint32_t* counter) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ uint32_t claimed;
  for (;;) {
    if (threadIdx.x == 0) claimed = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t it = claimed;
    __syncthreads();  // every wave has read `claimed` before it is written again
    if (it >= nitems) {  // uniform: every wave leaves together
      if (threadIdx.x == 0 && atomicAdd(counter + 1, 1u) == gridDim.x - 1) {
        atomicExch(counter, 0u);
        atomicExch(counter + 1, 0u);
      }
      break;
    }
    const WorkItem w = items[it];
    const GroupJob& job = jobs[w.group];
    if (job.kind == kJobResident) {
      if (job.rp.kparts > 1) resident_group_split<L>(job.rp, w.index, smem);
      else resident_group<L, false>(job.rp, w.index, smem);
    }
    else stream_block<L, uint32_t>(job.sp, w.index, smem);
    __syncthreads();  // LDS is reused by the next item
  }
}

}  // namespace pm

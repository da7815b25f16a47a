// ng_launch.hpp -- host-callable launchers of the HIP kernels (ng_kernels.hip).
// dim: 1 or 2; prec: 0 = FP64, 1 = FP32, 2 = mixed.  All launches are
// asynchronous on s.  Optional events e0 / e1 receive the kernel's own start
// and end (timed launches; never under stream capture).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ng_internal.hpp"

namespace ng {

// variant: 0 for any set of solves; 1 + r when every solve of the launch is
// periodic with the HLLC flux and closure recipe r (a kernel with that path
// only); kVariantCsph (dim 1, FP64) when every solve takes the CSPH-TVD step.
hipError_t launch_step(int dim, int prec, int variant, const InstDesc* descs, InstCtrl* ctrls,
                       const BlockRef* blocks, int64_t nblocks, int waves, int remap, int fused,
                       hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Priming pass: totals, checks and signal speed of the current state.  With
// blocks == nullptr the launch covers solve `inst`'s own workgroups 0..nblocks-1.
hipError_t launch_prime(int dim, int prec, const InstDesc* descs, InstCtrl* ctrls,
                        const BlockRef* blocks, int inst, int64_t nblocks, int waves,
                        hipStream_t s);
hipError_t launch_finalize(const InstDesc* descs, InstCtrl* ctrls, const int32_t* insts, int n,
                           int mode, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
hipError_t launch_small(int dim, int prec, const InstDesc* descs, InstCtrl* ctrls,
                        const int32_t* insts, int n, int waves, int64_t nsteps, hipStream_t s);
hipError_t launch_set_limits(InstCtrl* ctrls, const int32_t* insts, int n, double t_end,
                             int64_t max_steps_from_now, hipStream_t s);

// Cooperative launch of one 1D solve (solve `inst`) for up
// to nsteps <= kCoopMaxSteps steps: grid workgroups of `waves` waves, all
// resident together (the runtime refuses a grid that does not fit); cs is the
// batch's barrier block, cleared here first.  coop_capacity gives the
// resident workgroups per CU of that kernel and the largest waves per
// workgroup.  variant as for launch_step.
constexpr int64_t kCoopMaxSteps = int64_t(1) << 16;
hipError_t coop_capacity(int prec, int variant, int waves, int* blocks_per_cu, int* max_waves);
hipError_t launch_coop(int prec, int variant, const InstDesc* descs, InstCtrl* ctrls, int inst,
                       CoopSync* cs, int grid, int waves, int64_t nsteps, int32_t spin_limit,
                       hipStream_t s);

// Static scratch of the entry point that allocates nothing: its device
// address on the current device (looked up once per device), and the kernel
// that writes one solve's descriptor, control block, finalize index list and
// workgroup table into it.
constexpr size_t kStaticScratchBytes = size_t(2) << 20;
constexpr int kMaxDevices = 64;
hipError_t static_scratch(void** ptr);
hipError_t launch_static_setup(const InstDesc& d, const InstCtrl& c, InstDesc* descs,
                               InstCtrl* ctrls, int32_t* insts, BlockRef* blocks,
                               int64_t nblocks, hipStream_t s);

}  // namespace ng

// cg_kernels.hpp -- host-visible launchers of the HIP kernels.
#pragma once

#include "cg_device.hpp"

namespace cgd {

// Variants of the step kernel: KV_NSC carries the Navier-Stokes correction
// (Sec. 2.1.3; applied to the lattices whose descriptor has F_NSC, the others
// are stepped as by the plain variant), KV_ISO the second-neighbour colour
// gradient for every lattice of the launch.  KV_XCH (nearest-neighbour
// gradient only) is a launch choice, not a lattice property: wavefronts own
// whole 64-column blocks and take their edge columns from each other through
// LDS (full-line stores, for lattices beyond the cache), instead of holding
// halo columns in their own outer lanes.  Both give the same bits.
enum : int { KV_NSC = 1, KV_ISO = 2, KV_XCH = 4 };
// The variant a lattice needs alone.
inline int step_variant(const SlotDesc &d)
{
    return ((d.flags & F_NSC) ? KV_NSC : 0) | ((d.flags & F_ISO) ? KV_ISO : 0);
}
hipError_t launch_step(int storage, int tx, const SlotDesc *d, int nslots, int tiles, int parity, int idx,
                       hipStream_t s, int variant);
hipError_t launch_init(int storage, const SlotDesc *d, long long nodes, const float *fields, int which,
                       hipStream_t s);
int moments_blocks(long long nodes);
// Device scratch of lbm_diag_noalloc: room for the partial sums of
// kMaxMomentBlocks blocks (9 each) and the nine final sums.
constexpr int kMaxMomentBlocks = 2048;
constexpr size_t kScratchDoubles = (size_t)kMaxMomentBlocks * 9 + 9;
// Its address on the current device (looked up once per device).
hipError_t scratch_device_ptr(double **out);
hipError_t launch_moments(int storage, const SlotDesc *d, long long nodes, int parity, float *fields,
                          double *partial, double *out, const double *circle, hipStream_t s);
hipError_t launch_pops(int storage, const SlotDesc *d, long long nodes, int which, float *buf, bool get,
                       hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t n, hipStream_t s);

}  // namespace cgd

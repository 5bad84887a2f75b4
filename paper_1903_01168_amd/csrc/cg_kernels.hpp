// cg_kernels.hpp -- host-visible launchers of the HIP kernels.
#pragma once

#include "cg_device.hpp"

namespace cgd {

// nsc: launch the variant that carries the Navier-Stokes correction (Sec.
// 2.1.3); it applies the correction to the lattices whose descriptor has
// F_NSC and steps the others as the plain variant does
hipError_t launch_step(int storage, int tx, const SlotDesc *d, int nslots, int tiles, int parity, int idx,
                       hipStream_t s, bool nsc);
hipError_t launch_init(int storage, const SlotDesc *d, long long nodes, const float *fields, int which,
                       hipStream_t s);
int moments_blocks(long long nodes);
hipError_t launch_moments(int storage, const SlotDesc *d, long long nodes, int parity, float *fields,
                          double *partial, double *out, const double *circle, hipStream_t s);
hipError_t launch_pops(int storage, const SlotDesc *d, long long nodes, int which, float *buf, bool get,
                       hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t n, hipStream_t s);

}  // namespace cgd

// Stand-ins for the kernel launchers of the library, for a host-only build of the
// runtime (api.cpp) under sanitizers: the checks never reach a launch, and any that did
// would fail with an error instead of running a kernel.
#include "dsx_internal.h"

namespace dsx {
hipError_t launch_sums(const SumsParams&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fft_planes(const PlaneParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fft_axis1(const Axis1Params&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_recombine_nuclear(const RecombParams&, int, int, int, size_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_recombine_magnetic(const RecombParams&, int, int, size_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_recombine_direct(const RecombParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_recombine_magnetic_rows(const RecombParams&, int, size_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_bragg(const BraggParams&, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_dw_mean(const DwParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_lanczos(const LanczosParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_lanczos_points(const PointsParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_lanczos_stencil(const LanczosParams&, hipStream_t) { return hipErrorNotSupported; }
int recombine_max_threads(int, int) { return 512; }
size_t planes_lds_bytes(const PlaneParams&) { return 0; }
size_t axis1_lds_bytes(const Axis1Params&) { return 0; }
size_t lanczos_lds_bytes(const LanczosParams&) { return 0; }
}  // namespace dsx

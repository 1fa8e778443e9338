// The nuclear and folded recombination kernels for Taylor orders 0-4: explicit
// instantiations of their launchers (the kernels are defined in recombine.hip).  Kept in
// a unit of their own so that the orders compile in parallel.
#define DSX_RECOMBINE_PART 1
#include "recombine.hip"

namespace dsx {
template hipError_t launch_nuc_hc<0>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hc<1>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hc<2>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hc<3>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hc<4>(const RecombParams&, int, int, size_t, hipStream_t);
}  // namespace dsx

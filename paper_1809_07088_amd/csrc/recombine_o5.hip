// The nuclear and folded recombination kernels for Taylor orders 5-6: explicit
// instantiations of their launchers (the kernels are defined in recombine.hip).  Kept in
// a unit of their own so that the orders compile in parallel.
#define DSX_RECOMBINE_PART 1
#include "recombine.hip"

namespace dsx {
template hipError_t launch_nuc_hc<5>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hc<6>(const RecombParams&, int, int, size_t, hipStream_t);
}  // namespace dsx

// The nuclear and folded recombination kernels for Taylor orders 9-16: explicit
// instantiations of their launchers (the kernels are defined in recombine.hip).  Kept in
// a unit of their own so that the orders compile in parallel.
#define DSX_RECOMBINE_PART 1
#include "recombine.hip"

namespace dsx {
template hipError_t launch_nuc_hi<9>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hi<10>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hi<11>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hi<12>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hi<13>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hi<14>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hi<15>(const RecombParams&, int, int, size_t, hipStream_t);
template hipError_t launch_nuc_hi<16>(const RecombParams&, int, int, size_t, hipStream_t);
}  // namespace dsx

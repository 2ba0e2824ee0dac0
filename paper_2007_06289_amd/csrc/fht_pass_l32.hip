// Instantiates the FHT pass kernels for filter chunks of 32 samples (one translation unit per
// chunk length, so the library builds in parallel), and the persistent first-pass kernels.
#include "fht_pass_impl.h"

namespace fhtfbp {
template hipError_t launch_pass_l<32>(const PassArgs& a, int batch, hipStream_t stream);
template hipError_t launch_first_l<32>(const PassArgs& a, int grid, hipStream_t stream);
}  // namespace fhtfbp

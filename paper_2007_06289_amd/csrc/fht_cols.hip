// Column-tiled FHT passes (middle and last back-projection passes).
#include "fht_pass_impl.h"

namespace fhtfbp {

hipError_t launch_cols(const PassArgs& a, int batch, hipStream_t stream) {
  const int N = 1 << a.log2n;
  const int cblocks = N >> a.log2w;
  const size_t lds = cols_lds_bytes(a);
  const int threads = cols_threads(a);
  if (cols_classes(a) == 2)
    return launch_kernel(fht_cols_kernel<2>, a, batch * (N >> a.log2r) * cblocks, threads, lds,
                         stream);
  return launch_kernel(fht_cols_kernel<1>, a, batch * 4 * (N >> a.log2r) * cblocks, threads, lds,
                       stream);
}

}  // namespace fhtfbp

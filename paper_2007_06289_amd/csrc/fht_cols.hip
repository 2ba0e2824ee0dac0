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

// The last back-projection pass over 128 x 128 image tiles (5 levels, N >= 256).
hipError_t launch_image_tiles(const PassArgs& a, int batch, hipStream_t stream) {
  if (a.log2n < 8) return hipErrorInvalidValue;
  if (a.levels == 7) {
    // 7 levels: one 128-row strip per class at a time, 1024 threads
    PassArgs t = a;
    t.log2r = 7;
    t.log2w = 7;
    t.halo = 128;
    t.out_mode = OUT_IMG_V;
    const int tpr = (1 << a.log2n) >> 7;
    return launch_kernel(fht_image_tile7_kernel, t, batch * tpr * tpr, 1024,
                         kT7LdsFloats * sizeof(float), stream);
  }
  if (a.levels != 5) return hipErrorInvalidValue;
  PassArgs t = a;
  t.log2r = 5;
  t.log2w = 7;
  t.halo = 32;
  t.out_mode = OUT_IMG_V;
  const int tpr = (1 << a.log2n) >> 7;
  return launch_kernel(fht_image_tile_kernel, t, batch * tpr * tpr, 512,
                       kTileLdsFloats * sizeof(float), stream);
}

}  // namespace fhtfbp

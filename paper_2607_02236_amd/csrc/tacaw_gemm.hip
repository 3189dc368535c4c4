// DFT-as-GEMM chunk kernel on MFMA (split-precision operands). Placeholder
// until the kernel lands: reports the transform as unsupported.
#include "tacaw_internal.h"

namespace tacaw {

bool seg_gemm_supported(int) { return false; }
int seg_gemm_tile_pixels(int) { return 64; }
hipError_t launch_seg_gemm(int, int, bool, int, const SegArgs&, const void*, int, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace tacaw

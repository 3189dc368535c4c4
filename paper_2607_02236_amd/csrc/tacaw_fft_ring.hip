// Launchers of the ring-resident whole-series variant of the fused chunk kernel
// (deferred streaming: every frame of the launch's chunks is read from the ring, stored
// per frame or per pixel tile).
#include "seg_fft_kernel.h"

namespace tacaw {

template <int L, typename InT, bool SUB64>
static hipError_t launch_ring_t(const SegArgs& a, int n_tiles, hipStream_t st) {
  constexpr int NT = FftShape<L>::W * (L / FftShape<L>::N1);
  if (a.ring_tiles > 0) {
    if (a.n_det > 0)
      hipLaunchKernelGGL((seg_fft_kernel<L, InT, SUB64, true, 4>), dim3(n_tiles), dim3(NT), 0, st, a);
    else
      hipLaunchKernelGGL((seg_fft_kernel<L, InT, SUB64, false, 4>), dim3(n_tiles), dim3(NT), 0, st, a);
  } else {
    if (a.n_det > 0)
      hipLaunchKernelGGL((seg_fft_kernel<L, InT, SUB64, true, 2>), dim3(n_tiles), dim3(NT), 0, st, a);
    else
      hipLaunchKernelGGL((seg_fft_kernel<L, InT, SUB64, false, 2>), dim3(n_tiles), dim3(NT), 0, st, a);
  }
  return hipGetLastError();
}

template <int L>
static hipError_t launch_ring_l(int in_dtype, bool sub64, const SegArgs& a, int n_tiles,
                                hipStream_t st) {
  if (in_dtype == 1) return launch_ring_t<L, double2, true>(a, n_tiles, st);
  return sub64 ? launch_ring_t<L, float2, true>(a, n_tiles, st)
               : launch_ring_t<L, float2, false>(a, n_tiles, st);
}

hipError_t launch_seg_fft_ring(int L, int in_dtype, bool sub64, const SegArgs& a, int n_tiles,
                               hipStream_t st) {
  if (!a.from_ring || 2 * a.hop != L) return hipErrorInvalidValue;
  switch (L) {
    case 64: return launch_ring_l<64>(in_dtype, sub64, a, n_tiles, st);
    case 128: return launch_ring_l<128>(in_dtype, sub64, a, n_tiles, st);
    case 256: return launch_ring_l<256>(in_dtype, sub64, a, n_tiles, st);
    case 512: return launch_ring_l<512>(in_dtype, sub64, a, n_tiles, st);
    case 1024: return launch_ring_l<1024>(in_dtype, sub64, a, n_tiles, st);
    case 200: return launch_ring_l<200>(in_dtype, sub64, a, n_tiles, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace tacaw

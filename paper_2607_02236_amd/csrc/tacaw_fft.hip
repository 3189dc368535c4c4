// Launchers of the fused chunk kernel (push-buffer variants) and its shapes; the
// kernel itself is in seg_fft_kernel.h, the ring-resident variant is launched from
// tacaw_fft_ring.hip.
#include "seg_fft_kernel.h"

namespace tacaw {

template <int L, typename InT, bool SUB64, bool FULL>
static void launch_lean(const SegArgs& a, bool narrow, int n_tiles, hipStream_t st) {
  constexpr int NT = FftShape<L>::W * (L / FftShape<L>::N1);
  if (narrow) {
    if (a.n_det > 0)
      hipLaunchKernelGGL((seg_fft_kernel<L, InT, SUB64, true, 3, FULL>), dim3(n_tiles), dim3(NT), 0, st, a);
    else
      hipLaunchKernelGGL((seg_fft_kernel<L, InT, SUB64, false, 3, FULL>), dim3(n_tiles), dim3(NT), 0, st, a);
  } else {
    if (a.n_det > 0)
      hipLaunchKernelGGL((seg_fft_kernel<L, InT, SUB64, true, 1, FULL>), dim3(n_tiles), dim3(NT), 0, st, a);
    else
      hipLaunchKernelGGL((seg_fft_kernel<L, InT, SUB64, false, 1, FULL>), dim3(n_tiles), dim3(NT), 0, st, a);
  }
}

template <int L, typename InT, bool SUB64>
static hipError_t launch_t(const SegArgs& a, int n_tiles, hipStream_t st) {
  constexpr int NT = FftShape<L>::W * (L / FftShape<L>::N1);
  const bool lean = (2 * a.hop == L || a.hop == L) && !a.from_ring &&
                    (int64_t)a.s_lo * a.hop >= a.push_begin;
  // one descriptor per chunk when a chunk's frames span less than 2 GiB
  const int64_t span = pix_off((int64_t)a.n_k - 1, a.nx, a.row_stride) + 1;
  const bool narrow =
      ((int64_t)(L - 1) * a.fstride + span) * (int64_t)sizeof(InT) < ((int64_t)1 << 31);
  if (lean) {
    if (a.hop == L) launch_lean<L, InT, SUB64, true>(a, narrow, n_tiles, st);
    else launch_lean<L, InT, SUB64, false>(a, narrow, n_tiles, st);
  } else {
    if (a.n_det > 0)
      hipLaunchKernelGGL((seg_fft_kernel<L, InT, SUB64, true, 0>), dim3(n_tiles), dim3(NT), 0, st, a);
    else
      hipLaunchKernelGGL((seg_fft_kernel<L, InT, SUB64, false, 0>), dim3(n_tiles), dim3(NT), 0, st, a);
  }
  return hipGetLastError();
}

template <int L>
static hipError_t launch_l(int in_dtype, bool sub64, const SegArgs& a, int n_tiles,
                           hipStream_t st) {
  if (in_dtype == 1) return launch_t<L, double2, true>(a, n_tiles, st);
  return sub64 ? launch_t<L, float2, true>(a, n_tiles, st)
               : launch_t<L, float2, false>(a, n_tiles, st);
}

void seg_fft_split(int L, int* n1, int* n2) {
  int a = 0;
  switch (L) {
    case 64: a = FftShape<64>::N1; break;
    case 128: a = FftShape<128>::N1; break;
    case 256: a = FftShape<256>::N1; break;
    case 512: a = FftShape<512>::N1; break;
    case 1024: a = FftShape<1024>::N1; break;
    case 200: a = FftShape<200>::N1; break;
  }
  *n1 = a;
  *n2 = a ? L / a : 0;
}

bool seg_fft_supported(int L) {
  return L == 64 || L == 128 || L == 256 || L == 512 || L == 1024 || L == 200;
}

int seg_fft_tile_pixels(int L) {
  switch (L) {
    case 64: return FftShape<64>::W;
    case 128: return FftShape<128>::W;
    case 256: return FftShape<256>::W;
    case 512: return FftShape<512>::W;
    case 1024: return FftShape<1024>::W;
    case 200: return FftShape<200>::W;
  }
  return 0;
}

hipError_t launch_seg_fft(int L, int in_dtype, bool sub64, const SegArgs& a, int n_tiles,
                          hipStream_t st) {
  if (a.from_ring && 2 * a.hop == L) return launch_seg_fft_ring(L, in_dtype, sub64, a, n_tiles, st);
  switch (L) {
    case 64: return launch_l<64>(in_dtype, sub64, a, n_tiles, st);
    case 128: return launch_l<128>(in_dtype, sub64, a, n_tiles, st);
    case 256: return launch_l<256>(in_dtype, sub64, a, n_tiles, st);
    case 512: return launch_l<512>(in_dtype, sub64, a, n_tiles, st);
    case 1024: return launch_l<1024>(in_dtype, sub64, a, n_tiles, st);
    case 200: return launch_l<200>(in_dtype, sub64, a, n_tiles, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace tacaw

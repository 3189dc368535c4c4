// Plan runtime behind the C ABI declared in include/tacaw.h: descriptor
// validation (host only, before any HIP call), plan-owned device buffers,
// per-probe frame cursors and ring slots for streamed series, and the
// stream-ordered launch sequence of push / finalize / detector / backward.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tacaw.h"
#include "tacaw_internal.h"

using namespace tacaw;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int64_t kMaxDeviceBytes = (int64_t)260 << 30;  // refuse plans beyond HBM capacity
constexpr int kMaxTimed = 2;  // chunk launches per push (deferred mode: before and after the store)

enum MeanStrategy {
  kRefSampled = 0,     // c = windowed mean of frames sampled over the first chunk, exact
                       // correction at finalize (compact windows)
  kRefExactMean = 1,   // c = exact FP64 mean from a pre-pass over the whole series
  kRefZero = 2,        // c = 0 (mean NONE with a non-compact window)
};

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int64_t seg_count(int64_t frames, int L, int H) { return frames < L ? 0 : (frames - L) / H + 1; }

// Window values w(t), t = 0..L-1 in double precision.
std::vector<double> make_window(int kind, int L, double param) {
  std::vector<double> w(L, 1.0);
  for (int t = 0; t < L; ++t) {
    const double tt = t;
    switch (kind) {
      case TACAW_WIN_HANN:
        w[t] = 0.5 - 0.5 * std::cos(kTwoPi * tt / L);
        break;
      case TACAW_WIN_RECT:
        w[t] = 1.0;
        break;
      case TACAW_WIN_HANN_WIDTH: {
        const double d = tt - 0.5 * L, half = 0.5 * param * L;
        w[t] = std::fabs(d) <= half ? 0.5 + 0.5 * std::cos(kTwoPi * d / (param * L)) : 0.0;
        break;
      }
      case TACAW_WIN_TUKEY: {
        // periodic Tukey: symmetric Tukey of length L + 1 without its last sample;
        // the two cosine tapers together span alpha * L samples
        const double span = 0.5 * param * L;
        if (param <= 0.0) {
          w[t] = 1.0;
        } else if (tt < span) {
          w[t] = 0.5 * (1.0 - std::cos(M_PI * tt / span));
        } else if (tt > L - span) {
          w[t] = 0.5 * (1.0 - std::cos(M_PI * (L - tt) / span));
        } else {
          w[t] = 1.0;
        }
        break;
      }
    }
  }
  return w;
}

// d w / d r of the width-r Hann window
std::vector<double> make_window_dr(int L, double r) {
  std::vector<double> g(L, 0.0);
  for (int t = 0; t < L; ++t) {
    const double d = t - 0.5 * L;
    if (std::fabs(d) <= 0.5 * r * L) {
      const double ph = kTwoPi * d / (r * L);
      g[t] = 0.5 * std::sin(ph) * ph / r;
    }
  }
  return g;
}

uint16_t bf16_bits(float x) {  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}
uint16_t f16_bits(float x) {
  const _Float16 h = (_Float16)x;
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}
float f16_value(uint16_t b) {
  _Float16 h;
  std::memcpy(&h, &b, 2);
  return (float)h;
}

// Window-folded DFT matrix of the GEMM form as hi and lo 16-bit parts:
// [2][m_rows][2L], row 2r + c (c: 0 real, 1 imaginary part of output row r, which
// holds bin m = (r - roi_half) mod L), column 2t + c' (c' multiplies Re or Im of
// frame t): [[Fr, -Fi], [Fi, Fr]] interleaved; rows from 2 n_om on are zero.
std::vector<uint16_t> make_dft_matrix(const std::vector<double>& w, bool fp16, int n_om,
                                      int roi_half, int m_rows) {
  const int L = (int)w.size(), K2 = 2 * L;
  std::vector<uint16_t> out((size_t)2 * m_rows * K2, 0);
  for (int r = 0; r < n_om; ++r) {
    const int m = (r - roi_half + L) % L;
    for (int t = 0; t < L; ++t) {
      const double ang = -6.283185307179586476925286766559 * (double)(((int64_t)m * t) % L) / L;
      const double fr = w[t] * std::cos(ang), fi = w[t] * std::sin(ang);
      const double e[2][2] = {{fr, -fi}, {fi, fr}};
      for (int c = 0; c < 2; ++c) {
        for (int cp = 0; cp < 2; ++cp) {
          const double v = e[c][cp];
          const float vf = (float)v;
          uint16_t hi, lo;
          if (fp16) {
            hi = f16_bits(vf);
            lo = f16_bits((float)(v - (double)f16_value(hi)));
          } else {
            hi = bf16_bits(vf);
            lo = bf16_bits((float)(v - (double)bf16_value(hi)));
          }
          const size_t idx = (size_t)(2 * r + c) * K2 + (2 * t + cp);
          out[idx] = hi;
          out[(size_t)m_rows * K2 + idx] = lo;
        }
      }
    }
  }
  return out;
}

}  // namespace

// error state shared with the other translation units of the library
int tacaw::set_error(int code, const char* msg) { return fail(code, msg); }
void tacaw::clear_error() { g_err.clear(); }

struct tacaw_plan_s {
  tacaw_plan_desc d{};
  hipStream_t st = nullptr;
  int device = 0;
  int L = 0, H = 0, Ns = 0, n_k = 0, N1 = 0, N2 = 0, W = 0, n_tiles = 0;
  int n_om = 0, roi = 0, m_rows = 0;  // output rows, energy window M, GEMM rows
  int64_t n_used = 0;
  double sumw2 = 0.0;
  int n_corr = 0;
  int bins[kMaxCorr] = {0, 0, 0};  // correction bins 0, 1, L-1 and their output rows
  int rows[kMaxCorr] = {0, 0, 0};
  double2 wbin[kMaxCorr];
  std::vector<double> win;  // w(t), t = 0..L-1
  bool compact = false;
  int strategy = kRefSampled;
  int esz = 8;
  int state = 0;  // 0 open, 1 finalized
  int64_t dropped = 0;
  int n_pairs = 0;          // (tile, detector) pairs with a non-zero mask
  DetSlots det_slots{};
  int n_slots = 0;
  std::vector<int64_t> cursor;
  std::vector<int> slot_owner;
  std::vector<std::pair<void**, int64_t>> owned;
  int64_t bytes = 0;
  // device buffers
  float* win_t = nullptr;   // [N2][N1]
  float* dwin_t = nullptr;  // [N2][N1] (HANN_WIDTH)
  float2* tw = nullptr;     // [N2][N1]
  double2* cref = nullptr;  // [P][n_k]
  double2* msum = nullptr;  // [P][n_k]
  double2* xs = nullptr;    // [P][3][n_k]
  double2* pseg_tw = nullptr;    // per-chunk mean: [3][L] w(t) exp(-2 pi i bin t / L)
  double2* pseg_open = nullptr;  // per-chunk mean: [P][V][4][n_k] open chunk sums
  double* pcorr = nullptr;       // per-chunk mean: [P][3][n_k] sum_s |X_s(b)|^2
  double2* pref = nullptr;       // per-chunk mean: [P][n_k] reference of its FP64 sums
  double2* cmean = nullptr;      // per-chunk mean: [P][Ns][n_k] chunk means (for the adjoint)
  int pseg_V = 0;                // chunks that can hold one frame, ceil(L / H)
  double* S = nullptr;      // [n_om][n_k]
  double* masks = nullptr;  // [n_det][n_k]
  int32_t* pair_slot = nullptr;  // [n_tiles][n_det]
  double* Dp = nullptr;     // [n_det][P][n_om]
  double* dpart = nullptr;
  int64_t dpart_bytes = 0;
  void* ring = nullptr;
  void* fmat = nullptr;     // DFT-GEMM operand (GEMM transforms)
  double* scratch = nullptr;
  int64_t scratch_bytes = 0;
  float* gscale = nullptr;  // GEMM form: [P][n_k]
  double* qfac = nullptr;   // [n_om] quantum-statistics factor per row (temperature > 0)
  unsigned long long* nf = nullptr;  // non-finite count at finalize (TACAW_FLAG_CHECK_FINITE)
  int64_t nonfinite = 0;
  hipEvent_t ev[kMaxTimed][2] = {};  // chunk-kernel timing, up to kMaxTimed launches per push
  int n_timed = 0;                    // launches timed in the last push
  int64_t D = 0;                      // ring depth (frames per slot)
  int64_t rs = 0, span = 0;           // input pixel-row stride and elements spanned per frame
  bool deferred = false;              // deferred ring mode (ring_frames > seg_len)
  bool tiled = false;                 // the ring is stored per pixel tile
  std::vector<int> s_done;            // deferred mode: chunks processed per probe
  bool s_fresh = true;                // no chunk launch since the last reset: S is undefined
  bool ingest_open = false;           // tacaw_ingest_frames handed out ring rows
  int ingest_p0 = 0, ingest_np = 0;
  int64_t ingest_nf = 0;

  int alloc(void** p, int64_t bytes, const char* what) {
    if (bytes <= 0) {
      *p = nullptr;
      return TACAW_OK;
    }
    if (this->bytes + bytes > kMaxDeviceBytes)
      return fail(TACAW_ERR_OOM, std::string("plan would exceed device memory: ") + what);
    if (hipMalloc(p, (size_t)bytes) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return fail(TACAW_ERR_OOM, std::string("hipMalloc failed for ") + what);
    }
    this->bytes += bytes;
    owned.push_back({p, bytes});
    return TACAW_OK;
  }
  void release(void** p) {
    for (size_t i = 0; i < owned.size(); ++i) {
      if (owned[i].first == p) {
        if (*p) (void)hipFree(*p);
        bytes -= owned[i].second;
        *p = nullptr;
        owned.erase(owned.begin() + i);
        return;
      }
    }
  }
  ~tacaw_plan_s() {
    (void)hipStreamSynchronize(st);
    for (auto& o : owned)
      if (*o.first) (void)hipFree(*o.first);
    for (auto& e : ev)
      for (auto& x : e)
        if (x) (void)hipEventDestroy(x);
  }
};

static int hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(TACAW_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  }
  return TACAW_OK;
}

#define TRY(x)                  \
  do {                          \
    int _rc = (x);              \
    if (_rc != TACAW_OK) return _rc; \
  } while (0)

static bool transform_is_gemm(int t) { return t == TACAW_GEMM_BF16X3 || t == TACAW_GEMM_F16X3; }

// The per-chunk mean sums are formed in FP64 relative to a probe's first frame
// (they run on every push, before the chunk kernel fixes its own reference).
static RefSamples first_frame_sample() {
  RefSamples r{};
  r.n = 1;
  r.t[0] = 0;
  r.wt[0] = 1.0;
  r.inv_sum = 1.0;
  r.round32 = 0;
  return r;
}

// One chunk-kernel launch over chunks [s_lo, s_hi) of probes [probe0, probe0 + n_probes),
// followed by the per-probe detector partial reduce. from_ring: every frame is read from
// the ring (deferred mode); otherwise from the push buffer `src` (frame push_begin at its
// row 0) and, for frames before push_begin, from the ring.
static int run_chunks(tacaw_plan_t P, const void* src, int64_t pstride, int64_t fstride,
                      int64_t push_begin, bool from_ring, int probe0, int n_probes, int s_lo,
                      int s_hi) {
  SegArgs g{};
  g.in = src;
  g.pstride = pstride;
  g.fstride = fstride;
  g.nx = P->d.nx;
  g.row_stride = from_ring ? P->d.nx : P->rs;  // the ring holds contiguous frames
  g.push_begin = from_ring ? ((int64_t)1 << 62) : push_begin;
  g.ring = P->ring;
  g.ring_depth = P->D;
  g.ring_row_lo = (int32_t)(((int64_t)s_lo * P->H) % P->D);
  g.from_ring = from_ring ? 1 : 0;
  g.ring_tiles = P->tiled ? P->n_tiles : 0;
  g.n_slots = P->n_slots;
  g.n_k = P->n_k;
  g.probe0 = probe0;
  g.n_probes = n_probes;
  g.s_lo = s_lo;
  g.s_hi = s_hi;
  g.hop = P->H;
  g.track_mean = P->strategy == kRefSampled ? 1 : 0;
  g.corr_skip = P->pcorr ? 1 : 0;
  g.n_corr = P->n_corr;
  for (int b = 0; b < kMaxCorr; ++b) g.corr_rows[b] = P->rows[b];
  g.win_t = P->win_t;
  g.tw = P->tw;
  g.cref = P->cref;
  g.msum = P->msum;
  g.xs = P->xs;
  g.S = P->S;
  g.s_store = P->s_fresh ? 1 : 0;
  P->s_fresh = false;
  g.n_om = P->n_om;
  g.roi_half = P->roi;
  g.n_det = P->d.n_det;
  g.masks = P->masks;
  g.pair_slot = P->pair_slot;
  g.dpart = P->dpart;
  g.gscale = P->gscale;
  const bool sub64 = P->d.in_dtype == TACAW_C128 || P->strategy == kRefExactMean;
  const bool timed = P->n_timed < kMaxTimed && P->ev[0][0];
  if (timed) TRY(hip_check(hipEventRecord(P->ev[P->n_timed][0], P->st), "event"));
  if (transform_is_gemm(P->d.transform))
    TRY(hip_check(launch_seg_gemm(P->L, P->d.in_dtype, sub64,
                                  P->d.transform == TACAW_GEMM_F16X3 ? 1 : 0, g, P->fmat,
                                  P->m_rows, P->n_tiles, P->st),
                  "chunk GEMM kernel"));
  else
    TRY(hip_check(launch_seg_fft(P->L, P->d.in_dtype, sub64, g, P->n_tiles, P->st),
                  "chunk FFT kernel"));
  if (timed) {
    TRY(hip_check(hipEventRecord(P->ev[P->n_timed][1], P->st), "event"));
    ++P->n_timed;
  }
  if (P->d.n_det > 0 && P->n_pairs > 0)
    TRY(hip_check(launch_dpart_reduce(P->dpart, P->det_slots, n_probes, P->d.n_det, P->n_om,
                                      probe0, P->d.n_probe, P->Dp, P->st),
                  "detector partial reduce"));
  return TACAW_OK;
}

// Deferred mode, before frames [a, b) of a probe group enter the ring: completed
// chunks wait there until these rows would overwrite the oldest of them; then all
// completed chunks run in one launch.
static int deferred_make_room(tacaw_plan_t P, int probe0, int n_probes, int64_t a, int64_t b) {
  const int s_ready = (int)std::min<int64_t>(P->Ns, seg_count(a, P->L, P->H));
  const int sd = P->s_done[probe0];
  if (sd < s_ready && (int64_t)sd * P->H < b - P->D) {
    TRY(run_chunks(P, P->ring, 0, P->n_k, 0, true, probe0, n_probes, sd, s_ready));
    for (int i = 0; i < n_probes; ++i) P->s_done[probe0 + i] = s_ready;
  }
  return TACAW_OK;
}

// Deferred mode, after frames up to b are in the ring: at the end of the series
// the remaining chunks run.
static int deferred_finish(tacaw_plan_t P, int probe0, int n_probes, int64_t b) {
  const int sd = P->s_done[probe0];
  if (b >= P->n_used && sd < P->Ns) {
    TRY(run_chunks(P, P->ring, 0, P->n_k, 0, true, probe0, n_probes, sd, P->Ns));
    for (int i = 0; i < n_probes; ++i) P->s_done[probe0 + i] = P->Ns;
  }
  return TACAW_OK;
}

// Cursor and ring-slot bookkeeping after frames [a, b) of a probe group.
static void advance(tacaw_plan_t P, int probe0, int n_probes, int64_t a, int64_t b, bool ring_used) {
  for (int i = 0; i < n_probes; ++i) {
    const int p = probe0 + i, sl = p % P->n_slots;
    P->cursor[p] = b;
    if (b >= P->n_used) {
      if (P->slot_owner[sl] == p) P->slot_owner[sl] = -1;
    } else if (ring_used) {
      P->slot_owner[sl] = p;
    }
  }
  P->dropped += (int64_t)n_probes * std::max<int64_t>(0, b - std::max<int64_t>(a, P->n_used));
}

// Ring slots of a probe group are free or already theirs.
static int claim_slots(tacaw_plan_t P, int probe0, int n_probes) {
  if (n_probes > P->n_slots)
    return fail(TACAW_ERR_STATE, "ring capacity exceeded: more probes in flight than ring slots");
  for (int i = 0; i < n_probes; ++i) {
    const int p = probe0 + i, sl = p % P->n_slots;
    if (P->slot_owner[sl] != -1 && P->slot_owner[sl] != p)
      return fail(TACAW_ERR_STATE, "ring capacity exceeded: too many probes in flight");
  }
  if (!P->ring) {
    // tiled: whole tiles (the last one padded), zeroed once so that the padding
    // pixels, which no store writes, read as 0
    const int64_t px = P->tiled ? (int64_t)P->n_tiles * P->W : P->n_k;
    const int64_t rb = (int64_t)P->n_slots * P->D * px * P->esz;
    TRY(P->alloc(&P->ring, rb, "frame ring"));
    if (P->tiled) TRY(hip_check(launch_fill_zero(P->ring, rb, P->st), "ring padding"));
  }
  return TACAW_OK;
}

static int ensure_dpart(tacaw_plan_t P, int n_probes) {
  if (P->d.n_det == 0) return TACAW_OK;
  const int64_t need = (int64_t)std::max(P->n_pairs, 1) * n_probes * P->n_om * 8;
  if (need > P->dpart_bytes) {
    P->release((void**)&P->dpart);
    P->dpart_bytes = 0;
    TRY(P->alloc((void**)&P->dpart, need, "detector partials"));
    P->dpart_bytes = need;
  }
  return TACAW_OK;
}

extern "C" {

const char* tacaw_last_error(void) { return g_err.c_str(); }
const char* tacaw_version(void) { return "tacaw-mi355x 0.1"; }

int tacaw_read_probe(const void* d_buf, int64_t n_bytes, void* hip_stream, uint64_t* d_sum) {
  g_err.clear();
  if (!d_buf || !d_sum) return fail(TACAW_ERR_INVALID_ARG, "buffer and sum must not be NULL");
  if (n_bytes <= 0 || n_bytes % 16 != 0)
    return fail(TACAW_ERR_INVALID_ARG, "n_bytes must be a positive multiple of 16");
  if (((uintptr_t)d_buf) % 16 != 0 || ((uintptr_t)d_sum) % 8 != 0)
    return fail(TACAW_ERR_INVALID_ARG, "buffer must be 16-byte and sum 8-byte aligned");
  return hip_check(launch_read_probe(d_buf, n_bytes, d_sum, (hipStream_t)hip_stream), "read probe");
}

int tacaw_read_probe_columns(const void* d_buf, int64_t n_rows, int64_t row_bytes,
                             int32_t seg_bytes, void* hip_stream, uint64_t* d_sum) {
  g_err.clear();
  if (!d_buf || !d_sum) return fail(TACAW_ERR_INVALID_ARG, "buffer and sum must not be NULL");
  if (!(seg_bytes == 64 || seg_bytes == 128 || seg_bytes == 256 || seg_bytes == 512))
    return fail(TACAW_ERR_INVALID_ARG, "seg_bytes must be 64, 128, 256 or 512");
  if (n_rows < 1 || row_bytes < seg_bytes || row_bytes % seg_bytes != 0)
    return fail(TACAW_ERR_INVALID_ARG, "row_bytes must be a positive multiple of seg_bytes");
  if (row_bytes / seg_bytes > 65535)
    return fail(TACAW_ERR_INVALID_ARG, "at most 65535 columns");
  if (((uintptr_t)d_buf) % 8 != 0 || ((uintptr_t)d_sum) % 8 != 0)
    return fail(TACAW_ERR_INVALID_ARG, "buffer and sum must be 8-byte aligned");
  return hip_check(launch_read_probe_columns(d_buf, n_rows, row_bytes, seg_bytes, d_sum,
                                             (hipStream_t)hip_stream),
                   "column read probe");
}

int tacaw_plan_check(const tacaw_plan_desc* d) {
  g_err.clear();
  if (!d) return fail(TACAW_ERR_INVALID_ARG, "desc is NULL");
  if (d->n_probe < 1) return fail(TACAW_ERR_INVALID_ARG, "n_probe must be >= 1");
  if (d->ny < 1 || d->nx < 1) return fail(TACAW_ERR_INVALID_ARG, "ny and nx must be >= 1");
  if ((int64_t)d->ny * d->nx > (int64_t)1 << 30)
    return fail(TACAW_ERR_INVALID_ARG, "ny * nx must be <= 2^30");
  if (!((is_pow2(d->seg_len) && d->seg_len >= 64 && d->seg_len <= 1024) || d->seg_len == 200))
    return fail(TACAW_ERR_UNSUPPORTED, "seg_len must be a power of two in [64, 1024] or 200");
  if (!is_pow2(d->seg_len) && d->transform != TACAW_FFT_F32)
    return fail(TACAW_ERR_UNSUPPORTED, "seg_len 200 needs the FFT transform");
  if (d->hop < 1 || d->hop > d->seg_len)
    return fail(TACAW_ERR_INVALID_ARG, "hop must satisfy 1 <= hop <= seg_len");
  if (d->n_frames < d->seg_len)
    return fail(TACAW_ERR_INVALID_ARG, "n_frames must be >= seg_len (at least one full chunk)");
  if (d->window < TACAW_WIN_HANN || d->window > TACAW_WIN_CUSTOM)
    return fail(TACAW_ERR_INVALID_ARG, "unknown window");
  if (d->window == TACAW_WIN_CUSTOM && !d->h_window)
    return fail(TACAW_ERR_INVALID_ARG, "CUSTOM window needs h_window");
  if (!(d->temperature_K >= 0.0)) return fail(TACAW_ERR_INVALID_ARG, "temperature_K must be >= 0");
  if (d->window == TACAW_WIN_HANN_WIDTH && !(d->window_param > 0.0 && d->window_param <= 4.0))
    return fail(TACAW_ERR_INVALID_ARG, "HANN_WIDTH needs 0 < window_param <= 4");
  if (d->window == TACAW_WIN_TUKEY && !(d->window_param >= 0.0 && d->window_param <= 1.0))
    return fail(TACAW_ERR_INVALID_ARG, "TUKEY needs 0 <= alpha <= 1");
  if (d->mean_mode != TACAW_MEAN_GLOBAL && d->mean_mode != TACAW_MEAN_PER_SEGMENT && d->mean_mode != TACAW_MEAN_NONE)
    return fail(TACAW_ERR_INVALID_ARG, "unknown mean_mode");
  if (d->transform != TACAW_FFT_F32 && !transform_is_gemm(d->transform))
    return fail(TACAW_ERR_INVALID_ARG, "unknown transform");
  if (transform_is_gemm(d->transform) && !seg_gemm_supported(d->seg_len))
    return fail(TACAW_ERR_UNSUPPORTED, "GEMM transform does not support this seg_len");
  if (d->mean_mode == TACAW_MEAN_PER_SEGMENT) {
    if (d->transform == TACAW_GEMM_F16X3)
      return fail(TACAW_ERR_UNSUPPORTED,
                  "per-segment mean needs the FFT or bf16 GEMM transform (fp16 scales its "
                  "operands from the whole series)");
    if ((d->seg_len + d->hop - 1) / d->hop > kMaxPsegOpen)
      return fail(TACAW_ERR_UNSUPPORTED, "per-segment mean needs hop >= seg_len / 4");
    if (d->n_frames >= ((int64_t)1 << 31))
      return fail(TACAW_ERR_UNSUPPORTED, "per-segment mean needs n_frames < 2^31");
  }
  if (d->in_dtype != TACAW_C64 && d->in_dtype != TACAW_C128)
    return fail(TACAW_ERR_INVALID_ARG, "unknown in_dtype");
  if (d->probe_reduce != TACAW_PROBE_MEAN && d->probe_reduce != TACAW_PROBE_SUM)
    return fail(TACAW_ERR_INVALID_ARG, "unknown probe_reduce");
  if (!(d->dt_fs > 0.0)) return fail(TACAW_ERR_INVALID_ARG, "dt_fs must be > 0");
  if (d->n_det < 0 || d->n_det > kMaxDet) return fail(TACAW_ERR_INVALID_ARG, "n_det must be in [0, 8]");
  if (d->n_det > 0 && !d->d_masks) return fail(TACAW_ERR_INVALID_ARG, "n_det > 0 needs d_masks");
  if (d->max_probes_in_flight < 0 || d->max_probes_in_flight > d->n_probe)
    return fail(TACAW_ERR_INVALID_ARG, "max_probes_in_flight must be in [0, n_probe]");
  if (d->omega_half < 0 || d->omega_half > d->seg_len / 2 - 1)
    return fail(TACAW_ERR_INVALID_ARG, "omega_half must be in [0, seg_len/2 - 1]");
  if (d->k_row_stride != 0 && d->k_row_stride < d->nx)
    return fail(TACAW_ERR_INVALID_ARG, "k_row_stride must be 0 or >= nx");
  if (d->ring_frames != 0) {
    if (d->ring_frames <= d->seg_len || d->ring_frames % (d->seg_len / 2) != 0 ||
        d->ring_frames >= ((int64_t)1 << 30))
      return fail(TACAW_ERR_INVALID_ARG,
                  "ring_frames must be 0 or a multiple of seg_len/2 in (seg_len, 2^30)");
    if (d->transform == TACAW_GEMM_F16X3)
      return fail(TACAW_ERR_UNSUPPORTED,
                  "deferred ring mode needs the FFT or bf16 GEMM transform (fp16 scales its "
                  "operands from the whole series)");
  }
  if (d->flags & TACAW_FLAG_TILED_RING) {
    if (d->ring_frames == 0)
      return fail(TACAW_ERR_INVALID_ARG, "a tiled ring needs the deferred ring mode (ring_frames > 0)");
    if (2 * d->hop != d->seg_len)
      return fail(TACAW_ERR_UNSUPPORTED, "a tiled ring needs hop = seg_len / 2");
  }
  const int64_t n_k = (int64_t)d->ny * d->nx;
  const int64_t n_om = d->omega_half > 0 ? 2 * (int64_t)d->omega_half + 1 : d->seg_len;
  int64_t need = n_om * n_k * 8 + (int64_t)d->n_probe * n_k * 80 + (int64_t)d->n_det * n_k * 8;
  if (d->mean_mode == TACAW_MEAN_PER_SEGMENT)
    need += (int64_t)d->n_probe * n_k * (kMaxPsegOpen * (1 + kMaxCorr) * 16 + kMaxCorr * 8 +
                                         seg_count(d->n_frames, d->seg_len, d->hop) * 16);
  if (need > kMaxDeviceBytes) return fail(TACAW_ERR_OOM, "plan accumulators exceed device memory");
  return TACAW_OK;
}

int tacaw_plan(const tacaw_plan_desc* d, void* hip_stream, tacaw_plan_t* out) {
  if (!out) return fail(TACAW_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  TRY(tacaw_plan_check(d));
  tacaw_plan_s* P = new (std::nothrow) tacaw_plan_s();
  if (!P) return fail(TACAW_ERR_OOM, "host allocation failed");
  P->d = *d;
  P->st = (hipStream_t)hip_stream;
  P->L = d->seg_len;
  P->H = d->hop;
  P->Ns = (int)seg_count(d->n_frames, P->L, P->H);
  P->n_used = (int64_t)(P->Ns - 1) * P->H + P->L;
  P->n_k = d->ny * d->nx;
  P->esz = d->in_dtype == TACAW_C128 ? 16 : 8;
  P->roi = d->omega_half;
  P->n_om = P->roi > 0 ? 2 * P->roi + 1 : P->L;
  P->m_rows = (2 * P->n_om + 31) / 32 * 32;
  const bool gemm = transform_is_gemm(d->transform);
  P->W = gemm ? seg_gemm_tile_pixels(P->L, P->n_om) : seg_fft_tile_pixels(P->L);
  P->n_tiles = (P->n_k + P->W - 1) / P->W;
  P->cursor.assign(d->n_probe, 0);
  P->s_done.assign(d->n_probe, 0);
  P->deferred = d->ring_frames > 0;
  P->tiled = (d->flags & TACAW_FLAG_TILED_RING) != 0;
  P->rs = d->k_row_stride > 0 ? d->k_row_stride : d->nx;
  P->span = (int64_t)(d->ny - 1) * P->rs + d->nx;
  P->D = P->deferred ? d->ring_frames : P->L;
  P->n_slots = d->max_probes_in_flight > 0 ? d->max_probes_in_flight : d->n_probe;
  P->slot_owner.assign(P->n_slots, -1);

  // window, its DFT at every bin (FP64), and the correction bins
  std::vector<double> w = make_window(d->window, P->L, d->window_param);
  if (d->window == TACAW_WIN_CUSTOM) w.assign(d->h_window, d->h_window + P->L);
  P->win = w;
  P->sumw2 = 0.0;
  double sumw = 0.0;
  for (double x : w) {
    P->sumw2 += x * x;
    sumw += std::fabs(x);
  }
  if (!(P->sumw2 > 0.0)) {
    delete P;
    return fail(TACAW_ERR_INVALID_ARG, "window is identically zero");
  }
  std::vector<double2> Wm(P->L);
  for (int m = 0; m < P->L; ++m) {
    double re = 0.0, im = 0.0;
    for (int t = 0; t < P->L; ++t) {
      const double ang = -kTwoPi * (double)(((int64_t)m * t) % P->L) / P->L;
      re += w[t] * std::cos(ang);
      im += w[t] * std::sin(ang);
    }
    Wm[m] = make_double2(re, im);
  }
  auto tiny = [&](int m) { return std::hypot(Wm[m].x, Wm[m].y) <= 1e-9 * sumw; };
  bool only0 = true, only3 = true;
  for (int m = 1; m < P->L; ++m) {
    if (!tiny(m)) only0 = false;
    if (m != 1 && m != P->L - 1 && !tiny(m)) only3 = false;
  }
  P->compact = only0 || only3;
  P->n_corr = only0 ? 1 : (only3 ? 3 : 0);
  P->bins[0] = 0;
  P->bins[1] = 1;
  P->bins[2] = P->L - 1;
  for (int b = 0; b < kMaxCorr; ++b) P->rows[b] = (P->bins[b] + P->roi) % P->L;
  for (int b = 0; b < kMaxCorr; ++b) P->wbin[b] = Wm[P->bins[b]];
  if (gemm && (d->transform == TACAW_GEMM_F16X3 || !P->compact))
    // fp16 (its operand scale needs the whole series) and non-compact windows: the
    // exact mean (or zero) is subtracted before splitting
    P->strategy = d->mean_mode == TACAW_MEAN_GLOBAL ? kRefExactMean : kRefZero;
  else if (P->compact)
    P->strategy = kRefSampled;
  else
    P->strategy = d->mean_mode == TACAW_MEAN_GLOBAL ? kRefExactMean : kRefZero;

  if (d->mean_mode == TACAW_MEAN_PER_SEGMENT && P->strategy != kRefSampled) {
    delete P;
    return fail(TACAW_ERR_UNSUPPORTED,
                "per-segment mean needs a window whose DFT is confined to bins 0 and +-1");
  }
  if (P->deferred && P->strategy != kRefSampled) {
    delete P;
    return fail(TACAW_ERR_UNSUPPORTED,
                "deferred ring mode needs a window whose DFT is confined to bins 0 and +-1");
  }
  // FFT split L = N1 * N2 (tables are laid out per pass-1 thread)
  seg_fft_split(P->L, &P->N1, &P->N2);
  std::vector<float> wt(P->L), dwt(P->L);
  std::vector<float2> twt(P->L);
  const std::vector<double> dw =
      d->window == TACAW_WIN_HANN_WIDTH ? make_window_dr(P->L, d->window_param)
                                        : std::vector<double>(P->L, 0.0);
  for (int n2 = 0; n2 < P->N2; ++n2) {
    for (int n1 = 0; n1 < P->N1; ++n1) {
      const int t = P->N2 * n1 + n2;
      wt[n2 * P->N1 + n1] = (float)w[t];
      dwt[n2 * P->N1 + n1] = (float)dw[t];
      const int k1 = n1;
      const double ang = -kTwoPi * (double)(((int64_t)n2 * k1) % P->L) / P->L;
      twt[n2 * P->N1 + k1] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
  }

  int rc = TACAW_OK;
  auto A = [&](void** p, int64_t b, const char* what) {
    if (rc == TACAW_OK) rc = P->alloc(p, b, what);
  };
  if (hipGetDevice(&P->device) != hipSuccess) {
    (void)hipGetLastError();
    delete P;
    return fail(TACAW_ERR_HIP, "no HIP device available");
  }
  const int64_t nk = P->n_k, np = d->n_probe;
  A((void**)&P->win_t, P->L * 4, "window");
  A((void**)&P->dwin_t, P->L * 4, "window derivative");
  A((void**)&P->tw, P->L * 8, "twiddles");
  A((void**)&P->cref, np * nk * 16, "references");
  A((void**)&P->msum, np * nk * 16, "mean sums");
  A((void**)&P->xs, np * kMaxCorr * nk * 16, "correction sums");
  A((void**)&P->S, (int64_t)P->n_om * nk * 8, "spectrum accumulator");
  if (d->flags & TACAW_FLAG_CHECK_FINITE) A((void**)&P->nf, 8, "non-finite count");
  if (d->mean_mode == TACAW_MEAN_PER_SEGMENT) {
    P->pseg_V = (P->L + P->H - 1) / P->H;
    A((void**)&P->pseg_tw, (int64_t)kMaxCorr * P->L * 16, "per-chunk mean twiddles");
    A((void**)&P->pseg_open, np * P->pseg_V * (1 + kMaxCorr) * nk * 16, "open chunk sums");
    A((void**)&P->pcorr, np * kMaxCorr * nk * 8, "per-chunk mean corrections");
    A((void**)&P->pref, np * nk * 16, "per-chunk mean references");
    A((void**)&P->cmean, np * P->Ns * nk * 16, "chunk means");
  }
  A((void**)&P->scratch, 64, "scratch");
  if (d->temperature_K > 0.0) A((void**)&P->qfac, (int64_t)P->n_om * 8, "quantum factor");
  if (gemm) {
    A(&P->fmat, (int64_t)2 * P->m_rows * (2 * P->L) * 2, "DFT matrix");
    A((void**)&P->gscale, np * nk * 4, "operand scales");
  }
  if (d->n_det > 0) {
    A((void**)&P->masks, (int64_t)d->n_det * nk * 8, "masks");
    A((void**)&P->pair_slot, (int64_t)P->n_tiles * d->n_det * 4, "detector tile slots");
    A((void**)&P->Dp, (int64_t)d->n_det * np * P->n_om * 8, "per-probe detector spectra");
  }
  if (rc != TACAW_OK) {
    delete P;
    return rc;
  }
  auto H2D = [&](void* dst, const void* src, int64_t b) {
    if (rc == TACAW_OK) rc = hip_check(hipMemcpy(dst, src, (size_t)b, hipMemcpyHostToDevice), "upload");
  };
  H2D(P->win_t, wt.data(), P->L * 4);
  H2D(P->dwin_t, dwt.data(), P->L * 4);
  H2D(P->tw, twt.data(), P->L * 8);
  if (P->pseg_tw && rc == TACAW_OK) {
    std::vector<double2> pt((size_t)kMaxCorr * P->L, make_double2(0.0, 0.0));
    for (int b = 0; b < P->n_corr; ++b)
      for (int t = 0; t < P->L; ++t) {
        const double ang = -kTwoPi * (double)(((int64_t)P->bins[b] * t) % P->L) / P->L;
        pt[(size_t)b * P->L + t] = make_double2(w[t] * std::cos(ang), w[t] * std::sin(ang));
      }
    H2D(P->pseg_tw, pt.data(), (int64_t)pt.size() * 16);
  }
  if (P->qfac && rc == TACAW_OK) {
    // E_m = h nu_m, nu_m = m / (L dt) (m < L/2) or (m - L) / (L dt); factor x / (1 - e^-x),
    // x = E_m / (k_B T), limit 1 at E = 0
    const double h_ev_s = 6.62607015e-34 / 1.602176634e-19, kb_ev_k = 8.617333262e-5;
    std::vector<double> q(P->n_om);
    for (int r = 0; r < P->n_om; ++r) {
      const int m = (r - P->roi + P->L) % P->L;
      const int sm = m < (P->L + 1) / 2 ? m : m - P->L;
      const double e = h_ev_s * (double)sm / ((double)P->L * d->dt_fs * 1e-15);
      const double x = e / (kb_ev_k * d->temperature_K);
      q[r] = x == 0.0 ? 1.0 : x / (-std::expm1(-x));
    }
    H2D(P->qfac, q.data(), (int64_t)P->n_om * 8);
  }
  if (gemm && rc == TACAW_OK) {
    const std::vector<uint16_t> fm =
        make_dft_matrix(w, d->transform == TACAW_GEMM_F16X3, P->n_om, P->roi, P->m_rows);
    H2D(P->fmat, fm.data(), (int64_t)fm.size() * 2);
  }
  if (d->n_det > 0 && rc == TACAW_OK) {
    rc = hip_check(hipMemcpy(P->masks, d->d_masks, (size_t)d->n_det * nk * 8, hipMemcpyDeviceToDevice),
                   "mask copy");
    std::vector<double> hm((size_t)d->n_det * nk);
    if (rc == TACAW_OK)
      rc = hip_check(hipMemcpy(hm.data(), P->masks, hm.size() * 8, hipMemcpyDeviceToHost), "mask read");
    // one partial slot per (tile, detector) whose mask is non-zero on the tile,
    // numbered detector by detector so each detector's slots are contiguous
    std::vector<int32_t> slots((size_t)P->n_tiles * d->n_det, -1);
    int act = 0;
    for (int dd = 0; dd < d->n_det; ++dd) {
      P->det_slots.off[dd] = act;
      for (int t = 0; t < P->n_tiles; ++t) {
        const int64_t k1 = std::min<int64_t>(nk, (int64_t)(t + 1) * P->W);
        for (int64_t k = (int64_t)t * P->W; k < k1; ++k)
          if (hm[(size_t)dd * nk + k] != 0.0) {
            slots[(size_t)t * d->n_det + dd] = act++;
            break;
          }
      }
    }
    P->det_slots.off[d->n_det] = act;
    P->n_pairs = act;
    H2D(P->pair_slot, slots.data(), (int64_t)slots.size() * 4);
  }
  if (rc == TACAW_OK && (d->flags & TACAW_FLAG_TIME_KERNELS)) {
    for (auto& e : P->ev)
      for (auto& x : e)
        if (rc == TACAW_OK) rc = hip_check(hipEventCreate(&x), "event");
  }
  if (rc == TACAW_OK) rc = hip_check(hipDeviceSynchronize(), "plan setup");
  if (rc == TACAW_OK) {
    *out = P;
    rc = tacaw_reset(P);
    if (rc != TACAW_OK) {
      delete P;
      *out = nullptr;
    }
    return rc;
  }
  delete P;
  return rc;
}

int tacaw_reset(tacaw_plan_t P) {
  if (!P) return fail(TACAW_ERR_INVALID_ARG, "plan is NULL");
  const int64_t nk = P->n_k, np = P->d.n_probe;
  TRY(hip_check(launch_fill_zero(P->cref, np * nk * 16, P->st), "reset"));
  TRY(hip_check(launch_fill_zero(P->msum, np * nk * 16, P->st), "reset"));
  TRY(hip_check(launch_fill_zero(P->xs, np * kMaxCorr * nk * 16, P->st), "reset"));
  if (P->pcorr) {
    TRY(hip_check(launch_fill_zero(P->pseg_open, np * P->pseg_V * (1 + kMaxCorr) * nk * 16, P->st),
                  "reset"));
    TRY(hip_check(launch_fill_zero(P->pcorr, np * kMaxCorr * nk * 8, P->st), "reset"));
  }
  // S needs no zero fill: the first chunk launch after a reset writes every element
  if (P->Dp)
    TRY(hip_check(launch_fill_zero(P->Dp, (int64_t)P->d.n_det * np * P->n_om * 8, P->st), "reset"));
  std::fill(P->cursor.begin(), P->cursor.end(), 0);
  std::fill(P->s_done.begin(), P->s_done.end(), 0);
  P->s_fresh = true;
  P->ingest_open = false;
  std::fill(P->slot_owner.begin(), P->slot_owner.end(), -1);
  P->state = 0;
  P->dropped = 0;
  return TACAW_OK;
}

int tacaw_set_stream(tacaw_plan_t P, void* s) {
  if (!P) return fail(TACAW_ERR_INVALID_ARG, "plan is NULL");
  P->st = (hipStream_t)s;
  return TACAW_OK;
}

int tacaw_plan_get_info(tacaw_plan_t P, tacaw_plan_info* info) {
  if (!P || !info) return fail(TACAW_ERR_INVALID_ARG, "plan or info is NULL");
  std::memset(info, 0, sizeof(*info));
  info->n_segments = P->Ns;
  info->n_omega = P->n_om;
  info->frames_used = P->n_used;
  info->frames_dropped = P->dropped;
  info->device_bytes = P->bytes;
  info->state = P->state;
  int c = 0;
  for (int64_t x : P->cursor) c += x >= P->n_used;
  info->probes_complete = c;
  info->window_sum_sq = P->sumw2;
  info->tile_pixels = P->W;
  info->nonfinite = (int32_t)std::min<int64_t>(P->nonfinite, 0x7FFFFFFF);
  info->last_chunk_kernel_ms = -1.0;
  if (P->n_timed > 0) {
    double tot = 0.0;
    bool ok = true;
    for (int i = 0; i < P->n_timed && ok; ++i) {
      float ms = 0.0f;
      ok = hipEventSynchronize(P->ev[i][1]) == hipSuccess &&
           hipEventElapsedTime(&ms, P->ev[i][0], P->ev[i][1]) == hipSuccess;
      tot += ms;
    }
    if (ok)
      info->last_chunk_kernel_ms = tot;
    else
      (void)hipGetLastError();
  }
  return TACAW_OK;
}

void tacaw_destroy(tacaw_plan_t P) { delete P; }

// ---- checkpoint: the accumulator state at a probe boundary ----
namespace {
constexpr uint64_t kStateMagic = 0x31305354574154ull;  // "TAWTS01"
struct StateHeader {
  uint64_t magic;
  uint64_t fingerprint;  // of the descriptor fields the state depends on
  int64_t total_bytes;
  int32_t n_probe, n_k, n_om, n_det;
  int32_t per_chunk, s_defined;
  int64_t dropped;
};

// FNV-1a over the descriptor fields (no pointers or stream), the window values and
// the detector masks (copied back from the plan; synchronises its stream)
int state_fingerprint(tacaw_plan_s* P, uint64_t* out) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  };
  const tacaw_plan_desc& d = P->d;
  const int32_t tiled = (d.flags & TACAW_FLAG_TILED_RING) ? 1 : 0;
  mix(&d.n_probe, 4); mix(&d.ny, 4); mix(&d.nx, 4); mix(&d.n_frames, 8); mix(&d.seg_len, 4);
  mix(&d.hop, 4); mix(&d.window, 4); mix(&d.window_param, 8); mix(&d.mean_mode, 4);
  mix(&d.transform, 4); mix(&d.in_dtype, 4); mix(&d.probe_reduce, 4); mix(&d.n_det, 4);
  mix(&d.temperature_K, 8); mix(&d.ring_frames, 8); mix(&d.omega_half, 4); mix(&tiled, 4);
  mix(P->win.data(), P->win.size() * sizeof(double));
  if (P->d.n_det > 0) {
    std::vector<double> m((size_t)P->d.n_det * P->n_k);
    if (hipMemcpyAsync(m.data(), P->masks, m.size() * 8, hipMemcpyDeviceToHost, P->st) != hipSuccess ||
        hipStreamSynchronize(P->st) != hipSuccess) {
      (void)hipGetLastError();
      return fail(TACAW_ERR_HIP, "state fingerprint: mask copy failed");
    }
    mix(m.data(), m.size() * 8);
  }
  *out = h;
  return TACAW_OK;
}

// A device array of the state: [outer][n_probe][inner bytes] when per probe
// (outer x n_probe x inner = bytes), else one block of bytes.
struct StateArray {
  void* ptr;
  int64_t bytes;
  bool per_probe;
  int64_t outer, inner;
};

// the device arrays of the state, in order: S, references, mean sums, correction
// sums, per-probe detector spectra, and the per-chunk mean's corrections,
// references and chunk means
std::vector<StateArray> state_arrays(tacaw_plan_s* P) {
  const int64_t nk = P->n_k, np = P->d.n_probe;
  auto pp = [&](void* ptr, int64_t outer, int64_t inner) {
    return StateArray{ptr, outer * np * inner, true, outer, inner};
  };
  std::vector<StateArray> a = {
      StateArray{P->S, (int64_t)P->n_om * nk * 8, false, 0, 0},
      pp(P->cref, 1, nk * 16), pp(P->msum, 1, nk * 16), pp(P->xs, 1, kMaxCorr * nk * 16)};
  if (P->Dp) a.push_back(pp(P->Dp, P->d.n_det, (int64_t)P->n_om * 8));
  if (P->pcorr) {
    a.push_back(pp(P->pcorr, 1, kMaxCorr * nk * 8));
    a.push_back(pp(P->pref, 1, nk * 16));
    if (P->cmean) a.push_back(pp(P->cmean, 1, (int64_t)P->Ns * nk * 16));
  }
  return a;
}

int64_t state_bytes(tacaw_plan_s* P) {
  int64_t b = (int64_t)sizeof(StateHeader) + (int64_t)P->d.n_probe * 8;
  for (auto& x : state_arrays(P)) b += x.bytes;
  return b;
}

// every probe is untouched or complete, nothing in flight
bool at_probe_boundary(const tacaw_plan_s* P) {
  if (P->ingest_open) return false;
  for (int64_t c : P->cursor)
    if (c != 0 && c < P->n_used) return false;
  return true;
}
}  // namespace

int tacaw_plan_export(tacaw_plan_t P, void* h_buf, int64_t buf_bytes, int64_t* bytes_needed) {
  g_err.clear();
  if (!P) return fail(TACAW_ERR_INVALID_ARG, "plan is NULL");
  const int64_t need = state_bytes(P);
  if (bytes_needed) *bytes_needed = need;
  if (!h_buf) return TACAW_OK;
  if (buf_bytes < need) return fail(TACAW_ERR_SHAPE, "buffer smaller than the state");
  if (P->state != 0) return fail(TACAW_ERR_STATE, "plan is finalized");
  if (!at_probe_boundary(P))
    return fail(TACAW_ERR_STATE, "a probe is partially pushed: export at a probe boundary");
  StateHeader h{};
  h.magic = kStateMagic;
  TRY(state_fingerprint(P, &h.fingerprint));
  h.total_bytes = need;
  h.n_probe = P->d.n_probe;
  h.n_k = P->n_k;
  h.n_om = P->n_om;
  h.n_det = P->d.n_det;
  h.per_chunk = P->pcorr ? 1 : 0;
  h.s_defined = P->s_fresh ? 0 : 1;
  h.dropped = P->dropped;
  char* out = (char*)h_buf;
  std::memcpy(out, &h, sizeof h);
  out += sizeof h;
  std::memcpy(out, P->cursor.data(), (size_t)P->d.n_probe * 8);
  out += (int64_t)P->d.n_probe * 8;
  const auto arrays = state_arrays(P);
  std::vector<char*> at;
  for (auto& x : arrays) {
    at.push_back(out);
    if (x.ptr == P->S && P->s_fresh) {
      std::memset(out, 0, (size_t)x.bytes);  // no chunk launched since the reset
    } else {
      TRY(hip_check(hipMemcpyAsync(out, x.ptr, (size_t)x.bytes, hipMemcpyDeviceToHost, P->st),
                    "state export"));
    }
    out += x.bytes;
  }
  TRY(hip_check(hipStreamSynchronize(P->st), "state export"));
  // an untouched probe's entries are zero in every array (some per-probe buffers
  // are only written when the probe runs), so that states of disjoint probe sets
  // add up to their union
  const int64_t np = P->d.n_probe;
  for (size_t i = 0; i < arrays.size(); ++i) {
    if (!arrays[i].per_probe) continue;
    for (int64_t p = 0; p < np; ++p) {
      if (P->cursor[(size_t)p] != 0) continue;
      for (int64_t o = 0; o < arrays[i].outer; ++o)
        std::memset(at[i] + (o * np + p) * arrays[i].inner, 0, (size_t)arrays[i].inner);
    }
  }
  return TACAW_OK;
}

int tacaw_state_merge(const void* h_a, const void* h_b, void* h_out, int64_t bytes) {
  g_err.clear();
  if (!h_a || !h_b || !h_out) return fail(TACAW_ERR_INVALID_ARG, "states must not be NULL");
  if (bytes < (int64_t)sizeof(StateHeader)) return fail(TACAW_ERR_SHAPE, "state buffer too small");
  StateHeader ha, hb;
  std::memcpy(&ha, h_a, sizeof ha);
  std::memcpy(&hb, h_b, sizeof hb);
  if (ha.magic != kStateMagic || hb.magic != kStateMagic)
    return fail(TACAW_ERR_INVALID_ARG, "not a plan state");
  if (ha.fingerprint != hb.fingerprint || ha.total_bytes != hb.total_bytes ||
      ha.n_probe != hb.n_probe || ha.n_k != hb.n_k || ha.n_om != hb.n_om ||
      ha.n_det != hb.n_det || ha.per_chunk != hb.per_chunk)
    return fail(TACAW_ERR_SHAPE, "the states belong to plans with different descriptors");
  if (ha.total_bytes != bytes || ha.n_probe < 1 ||
      (int64_t)sizeof(StateHeader) + (int64_t)ha.n_probe * 8 > bytes ||
      (bytes - (int64_t)sizeof(StateHeader) - (int64_t)ha.n_probe * 8) % 8 != 0)
    return fail(TACAW_ERR_SHAPE, "state size does not match its header");
  const int64_t np = ha.n_probe;
  std::vector<int64_t> ca((size_t)np), cb((size_t)np);
  std::memcpy(ca.data(), (const char*)h_a + sizeof ha, (size_t)np * 8);
  std::memcpy(cb.data(), (const char*)h_b + sizeof hb, (size_t)np * 8);
  for (int64_t p = 0; p < np; ++p)
    if (ca[p] != 0 && cb[p] != 0)
      return fail(TACAW_ERR_INVALID_ARG,
                  "probe " + std::to_string(p) + " was pushed in both states");
  // every accumulator is a sum over probes and chunks, and each probe's own entries
  // are zero where it was not pushed: the union is the element-wise FP64 sum
  const int64_t n = (bytes - (int64_t)sizeof(StateHeader) - np * 8) / 8;
  const double* xa = (const double*)((const char*)h_a + sizeof ha + np * 8);
  const double* xb = (const double*)((const char*)h_b + sizeof hb + np * 8);
  std::vector<double> sum((size_t)n);
  for (int64_t i = 0; i < n; ++i) sum[(size_t)i] = xa[i] + xb[i];
  StateHeader ho = ha;
  ho.s_defined = ha.s_defined | hb.s_defined;
  ho.dropped = ha.dropped + hb.dropped;
  char* out = (char*)h_out;  // may alias h_a or h_b: everything was read above
  std::memcpy(out, &ho, sizeof ho);
  for (int64_t p = 0; p < np; ++p) ca[p] = ca[p] != 0 ? ca[p] : cb[p];
  std::memcpy(out + sizeof ho, ca.data(), (size_t)np * 8);
  std::memcpy(out + sizeof ho + np * 8, sum.data(), (size_t)n * 8);
  return TACAW_OK;
}

int tacaw_plan_import(tacaw_plan_t P, const void* h_buf, int64_t bytes) {
  g_err.clear();
  if (!P || !h_buf) return fail(TACAW_ERR_INVALID_ARG, "plan and buffer must not be NULL");
  if (P->state != 0 || P->ingest_open)
    return fail(TACAW_ERR_STATE, "import into an open plan with nothing in flight");
  for (int64_t c : P->cursor)
    if (c != 0) return fail(TACAW_ERR_STATE, "import into a plan with no frames pushed");
  if (bytes < (int64_t)sizeof(StateHeader)) return fail(TACAW_ERR_SHAPE, "state buffer too small");
  StateHeader h;
  std::memcpy(&h, h_buf, sizeof h);
  if (h.magic != kStateMagic) return fail(TACAW_ERR_INVALID_ARG, "not a plan state");
  uint64_t fp = 0;
  TRY(state_fingerprint(P, &fp));
  if (h.fingerprint != fp || h.n_probe != P->d.n_probe || h.n_k != P->n_k ||
      h.n_om != P->n_om || h.n_det != P->d.n_det || h.per_chunk != (P->pcorr ? 1 : 0))
    return fail(TACAW_ERR_SHAPE, "the state belongs to a plan with another descriptor");
  const int64_t need = state_bytes(P);
  if (h.total_bytes != need || bytes < need) return fail(TACAW_ERR_SHAPE, "state buffer truncated");
  const char* in = (const char*)h_buf + sizeof h;
  std::vector<int64_t> cur((size_t)P->d.n_probe);
  std::memcpy(cur.data(), in, (size_t)P->d.n_probe * 8);
  in += (int64_t)P->d.n_probe * 8;
  for (int64_t c : cur)
    if (c < 0 || (c != 0 && c < P->n_used) || c > P->d.n_frames)
      return fail(TACAW_ERR_INVALID_ARG, "state holds a probe cursor off a probe boundary");
  for (auto& x : state_arrays(P)) {
    TRY(hip_check(hipMemcpyAsync(x.ptr, in, (size_t)x.bytes, hipMemcpyHostToDevice, P->st),
                  "state import"));
    in += x.bytes;
  }
  TRY(hip_check(hipStreamSynchronize(P->st), "state import"));
  for (int p = 0; p < P->d.n_probe; ++p) {
    P->cursor[p] = cur[p];
    P->s_done[p] = cur[p] >= P->n_used ? P->Ns : 0;
  }
  P->s_fresh = h.s_defined == 0;
  P->dropped = h.dropped;
  return TACAW_OK;
}

// Per-chunk mean: stream frames [a, min(b, n_used)) of a push through the FP64
// chunk sums (after the references exist).
static int run_pseg(tacaw_plan_t P, const void* frames, int64_t pstride, int64_t fstride,
                    int64_t rs, int32_t probe0, int32_t n_probes, int64_t a, int64_t b) {
  PsegArgs g{};
  g.in = frames;
  g.pstride = pstride;
  g.fstride = fstride;
  g.rs = rs;
  g.nx = P->d.nx;
  g.n_k = P->n_k;
  g.probe0 = probe0;
  g.n_probes = n_probes;
  g.base = a;
  g.f_lo = a;
  g.f_hi = std::min<int64_t>(b, P->n_used);
  g.L = P->L;
  g.H = P->H;
  g.Ns = P->Ns;
  g.n_corr = P->n_corr;
  g.V = P->pseg_V;
  for (int i = 0; i < kMaxCorr; ++i) g.wbin[i] = P->wbin[i];
  g.tw = P->pseg_tw;
  g.cref = P->pref;
  g.open = P->pseg_open;
  g.pcorr = P->pcorr;
  g.cmean = P->cmean;
  return hip_check(launch_pseg(g, P->d.in_dtype, P->st), "per-chunk mean sums");
}

int tacaw_push_frames(tacaw_plan_t P, const void* frames, int32_t probe0, int32_t n_probes,
                      int64_t n_frames, int64_t pstride, int64_t fstride) {
  g_err.clear();
  if (!P) return fail(TACAW_ERR_INVALID_ARG, "plan is NULL");
  if (P->state != 0) return fail(TACAW_ERR_STATE, "plan is finalized");
  if (P->ingest_open) return fail(TACAW_ERR_STATE, "an ingest is open: commit it first");
  if (n_frames < 0) return fail(TACAW_ERR_INVALID_ARG, "n_frames must be >= 0");
  if (n_probes < 1 || probe0 < 0 || probe0 + (int64_t)n_probes > P->d.n_probe)
    return fail(TACAW_ERR_SHAPE, "probe range outside the plan");
  if (n_frames == 0) return TACAW_OK;
  if (!frames) return fail(TACAW_ERR_INVALID_ARG, "frames is NULL");
  if (((uintptr_t)frames) % P->esz != 0)
    return fail(TACAW_ERR_INVALID_ARG, "frames pointer is not aligned to its element size");
  if (fstride < P->span)
    return fail(TACAW_ERR_INVALID_ARG, "frame_stride must cover a frame ((ny - 1) * row stride + nx)");
  if (n_probes > 1 && pstride < 1) return fail(TACAW_ERR_INVALID_ARG, "probe_stride must be >= 1");
  if (((int64_t)P->N2 * fstride + P->span) * P->esz > (int64_t)0x7FFFFFFFLL)
    return fail(TACAW_ERR_UNSUPPORTED, "frame_stride too large for 31-bit row-group offsets");
  const int64_t a = P->cursor[probe0];
  for (int i = 1; i < n_probes; ++i)
    if (P->cursor[probe0 + i] != a)
      return fail(TACAW_ERR_STATE, "probes of one push must be at the same frame cursor");
  const int64_t b = a + n_frames;
  if (b > P->d.n_frames) return fail(TACAW_ERR_SHAPE, "push goes beyond the plan's n_frames");
  // the exact-mean pre-pass, the fp16 operand scale and the GEMM form without the
  // streaming reference read each probe's whole series at once
  if ((P->strategy == kRefExactMean ||
       (transform_is_gemm(P->d.transform) && P->strategy != kRefSampled)) &&
      (a != 0 || b < P->n_used))
    return fail(TACAW_ERR_UNSUPPORTED,
                "this plan needs each probe's whole series in one push (exact mean pre-pass)");

  const int s_lo = (int)std::min<int64_t>(P->Ns, seg_count(a, P->L, P->H));
  const int s_hi = (int)std::min<int64_t>(P->Ns, seg_count(b, P->L, P->H));
  if (P->deferred) {
    if (n_frames > P->D - P->L)
      return fail(TACAW_ERR_SHAPE, "in deferred mode a push may hold at most ring_frames - seg_len frames");
    for (int i = 1; i < n_probes; ++i)
      if (P->s_done[probe0 + i] != P->s_done[probe0])
        return fail(TACAW_ERR_STATE, "probes of one push must have processed the same chunks");
  }
  // frames later chunks still need after this push (immediate mode)
  const int64_t keep_lo = std::max<int64_t>(a, (int64_t)s_hi * P->H);
  const int64_t keep_hi = std::min<int64_t>(b, P->n_used);
  const bool need_ring_write = P->deferred ? a < P->n_used : (s_hi < P->Ns && keep_hi > keep_lo);
  const bool need_ring_read = P->deferred || (s_hi > s_lo && (int64_t)s_lo * P->H < a);
  if (need_ring_write || need_ring_read) TRY(claim_slots(P, probe0, n_probes));
  TRY(ensure_dpart(P, n_probes));

  // 1. references: the chunk kernel fixes a kRefSampled reference from the probe's
  // first chunk; the per-chunk mean sums take the first frame
  if (a == 0) {
    if (P->pref)
      TRY(hip_check(launch_ref_sampled(frames, P->d.in_dtype, pstride, fstride, P->d.nx, P->rs,
                                       first_frame_sample(), probe0, n_probes, P->n_k, P->pref,
                                       P->st),
                    "reference"));
    if (P->strategy == kRefExactMean)
      TRY(hip_check(launch_ref_mean(frames, P->d.in_dtype, pstride, fstride, P->d.nx, P->rs,
                                    P->n_used, probe0, n_probes, P->n_k, P->cref, P->st),
                    "mean pre-pass"));
    if (P->d.transform == TACAW_GEMM_F16X3)
      TRY(hip_check(launch_gemm_scale(frames, P->d.in_dtype, pstride, fstride, P->d.nx, P->rs,
                                      P->n_used, probe0, n_probes, P->n_k,
                                      P->d.transform == TACAW_GEMM_F16X3 ? 1 : 0, P->cref,
                                      P->gscale, P->st),
                    "operand scale pre-pass"));
  }
  if (P->pcorr) TRY(run_pseg(P, frames, pstride, fstride, P->rs, probe0, n_probes, a, b));
  P->n_timed = 0;
  if (!P->deferred) {
    // 2. every chunk completed by this push, read from the push (and the ring)
    if (s_hi > s_lo) TRY(run_chunks(P, frames, pstride, fstride, a, false, probe0, n_probes, s_lo, s_hi));
    // 3. keep what later chunks need
    if (need_ring_write)
      TRY(hip_check(launch_ring_store(frames, P->d.in_dtype, pstride, fstride, P->d.nx, P->rs, a,
                                      keep_lo, keep_hi, probe0, n_probes, P->n_slots, P->D,
                                      P->n_k, 0, P->ring, P->st),
                    "ring store"));
  } else {
    // deferred: the push is copied into the ring; completed chunks run from there
    TRY(deferred_make_room(P, probe0, n_probes, a, b));
    if (need_ring_write)
      TRY(hip_check(launch_ring_store(frames, P->d.in_dtype, pstride, fstride, P->d.nx, P->rs, a,
                                      a, std::min<int64_t>(b, P->n_used), probe0, n_probes,
                                      P->n_slots, P->D, P->n_k, P->tiled ? P->W : 0, P->ring,
                                      P->st),
                    "ring store"));
    TRY(deferred_finish(P, probe0, n_probes, b));
  }
  advance(P, probe0, n_probes, a, b, need_ring_write || need_ring_read);
  return TACAW_OK;
}

// Ring rows for the next n_frames frames of probes [probe0, probe0 + n_probes)
// (deferred mode); chunks that would be overwritten run first.
static int ingest_rows(tacaw_plan_t P, int32_t probe0, int32_t n_probes, int64_t n_frames,
                       bool tiled, int64_t* slot0, int64_t* row0) {
  if (P->state != 0) return fail(TACAW_ERR_STATE, "plan is finalized");
  if (!P->deferred) return fail(TACAW_ERR_STATE, "ingest needs the deferred ring mode");
  if (P->tiled != tiled)
    return fail(TACAW_ERR_STATE, tiled ? "tiled ingest needs TACAW_FLAG_TILED_RING"
                                       : "ingest needs the per-frame ring layout (no TACAW_FLAG_TILED_RING)");
  if (tiled && P->pcorr)
    return fail(TACAW_ERR_STATE, "the per-chunk mean reads per-frame rows: no tiled ingest");
  if (P->ingest_open) return fail(TACAW_ERR_STATE, "the previous ingest is not committed");
  if (n_probes < 1 || probe0 < 0 || probe0 + (int64_t)n_probes > P->d.n_probe)
    return fail(TACAW_ERR_SHAPE, "probe range outside the plan");
  if (n_frames < 1 || n_frames > P->D - P->L)
    return fail(TACAW_ERR_SHAPE, "an ingest holds 1 .. ring_frames - seg_len frames");
  const int64_t a = P->cursor[probe0], b = a + n_frames;
  for (int i = 1; i < n_probes; ++i)
    if (P->cursor[probe0 + i] != a || P->s_done[probe0 + i] != P->s_done[probe0])
      return fail(TACAW_ERR_STATE, "probes of one ingest must be at the same frame cursor");
  if (b > P->n_used) return fail(TACAW_ERR_SHAPE, "ingest goes beyond the frames the chunks use");
  if (a % P->D + n_frames > P->D)
    return fail(TACAW_ERR_SHAPE, "ingest would wrap around the ring (align pieces to ring_frames)");
  if (probe0 % P->n_slots + n_probes > P->n_slots)
    return fail(TACAW_ERR_SHAPE, "ingest probes must occupy consecutive ring slots");
  TRY(claim_slots(P, probe0, n_probes));
  TRY(ensure_dpart(P, n_probes));
  P->n_timed = 0;  // the chunk launches of this ingest and its commit are timed together
  TRY(deferred_make_room(P, probe0, n_probes, a, b));
  *slot0 = probe0 % P->n_slots;
  *row0 = a % P->D;
  P->ingest_open = true;
  P->ingest_p0 = probe0;
  P->ingest_np = n_probes;
  P->ingest_nf = n_frames;
  return TACAW_OK;
}

int tacaw_ingest_frames(tacaw_plan_t P, int32_t probe0, int32_t n_probes, int64_t n_frames,
                        void** d_dst, int64_t* probe_stride, int64_t* frame_stride) {
  g_err.clear();
  if (!P || !d_dst || !probe_stride || !frame_stride)
    return fail(TACAW_ERR_INVALID_ARG, "plan and output pointers must not be NULL");
  *d_dst = nullptr;
  int64_t slot0 = 0, row0 = 0;
  TRY(ingest_rows(P, probe0, n_probes, n_frames, false, &slot0, &row0));
  *d_dst = (char*)P->ring + ((slot0 * P->D + row0) * P->n_k) * P->esz;
  *probe_stride = P->D * P->n_k;
  *frame_stride = P->n_k;
  return TACAW_OK;
}

int tacaw_ingest_frames_tiled(tacaw_plan_t P, int32_t probe0, int32_t n_probes,
                              int64_t n_frames, void** d_dst, int64_t* probe_stride,
                              int64_t* frame_stride, int64_t* tile_stride, int32_t* tile_pixels) {
  g_err.clear();
  if (!P || !d_dst || !probe_stride || !frame_stride || !tile_stride || !tile_pixels)
    return fail(TACAW_ERR_INVALID_ARG, "plan and output pointers must not be NULL");
  *d_dst = nullptr;
  int64_t slot0 = 0, row0 = 0;
  TRY(ingest_rows(P, probe0, n_probes, n_frames, true, &slot0, &row0));
  // ring [slot][tile][row][W]
  *d_dst = (char*)P->ring + (((slot0 * P->n_tiles) * P->D + row0) * P->W) * P->esz;
  *probe_stride = (int64_t)P->n_tiles * P->D * P->W;
  *tile_stride = P->D * P->W;
  *frame_stride = P->W;
  *tile_pixels = P->W;
  return TACAW_OK;
}

int tacaw_commit_frames(tacaw_plan_t P, int32_t probe0, int32_t n_probes, int64_t n_frames) {
  g_err.clear();
  if (!P) return fail(TACAW_ERR_INVALID_ARG, "plan is NULL");
  if (!P->ingest_open || P->ingest_p0 != probe0 || P->ingest_np != n_probes ||
      P->ingest_nf != n_frames)
    return fail(TACAW_ERR_STATE, "commit does not match the open ingest");
  P->ingest_open = false;
  const int64_t a = P->cursor[probe0], b = a + n_frames;
  if (a == 0 && P->pref) {  // the per-chunk sums' reference: frame 0, now in the ring
    const int64_t slot0 = probe0 % P->n_slots;
    TRY(hip_check(launch_ref_sampled((char*)P->ring + slot0 * P->D * P->n_k * P->esz,
                                     P->d.in_dtype, P->D * P->n_k, P->n_k, P->d.nx, P->d.nx,
                                     first_frame_sample(), probe0, n_probes, P->n_k, P->pref,
                                     P->st),
                  "reference"));
  }
  if (P->pcorr) {
    const int64_t slot0 = probe0 % P->n_slots;
    TRY(run_pseg(P, (char*)P->ring + ((slot0 * P->D + a % P->D) * P->n_k) * P->esz,
                 P->D * P->n_k, P->n_k, P->d.nx, probe0, n_probes, a, b));
  }
  TRY(deferred_finish(P, probe0, n_probes, b));
  advance(P, probe0, n_probes, a, b, true);
  return TACAW_OK;
}

static CorrArgs corr_args(tacaw_plan_t P) {
  CorrArgs c{};
  c.n_k = P->n_k;
  c.n_probe = P->d.n_probe;
  c.n_om = P->n_om;
  c.n_corr = P->n_corr;
  c.mean_global = P->d.mean_mode == TACAW_MEAN_GLOBAL ? 1 : 0;
  for (int b = 0; b < kMaxCorr; ++b) {
    c.rows[b] = P->rows[b];
    c.wbin[b] = P->wbin[b];
  }
  c.inv_nused = 1.0 / (double)P->n_used;
  c.n_seg = (double)P->Ns;
  c.cref = P->cref;
  c.msum = P->msum;
  c.xs = P->xs;
  c.pcorr = P->pcorr;
  return c;
}

static double kappa_probe(tacaw_plan_t P) { return 1.0 / ((double)P->L * P->sumw2 * (double)P->Ns); }
static double kappa_S(tacaw_plan_t P) {
  return kappa_probe(P) / (P->d.probe_reduce == TACAW_PROBE_MEAN ? (double)P->d.n_probe : 1.0);
}

int tacaw_finalize(tacaw_plan_t P, double* d_S) {
  g_err.clear();
  if (!P) return fail(TACAW_ERR_INVALID_ARG, "plan is NULL");
  if (P->state != 0) return fail(TACAW_ERR_STATE, "plan is already finalized");
  if (P->ingest_open) return fail(TACAW_ERR_STATE, "an ingest is open: commit it first");
  for (int p = 0; p < P->d.n_probe; ++p)
    if (P->cursor[p] < P->n_used)
      return fail(TACAW_ERR_STATE, "series incomplete for probe " + std::to_string(p));
  if (P->strategy == kRefSampled) {
    const CorrArgs c = corr_args(P);
    TRY(hip_check(launch_correct_S(c, P->S, nullptr, 0.0, P->st), "mean correction"));
    if (P->d.n_det > 0)
      TRY(hip_check(launch_correct_Dp(c, P->masks, P->d.n_det, P->Dp, P->st), "mean correction"));
  }
  TRY(hip_check(launch_finalize_S(P->S, d_S, (int64_t)P->n_om * P->n_k, kappa_S(P), P->qfac,
                                  P->n_k, P->n_om, P->st),
                "normalisation"));
  if (P->d.n_det > 0)
    TRY(hip_check(launch_finalize_S(P->Dp, nullptr, (int64_t)P->d.n_det * P->d.n_probe * P->n_om,
                                    kappa_probe(P), P->qfac, 1, P->n_om, P->st),
                  "normalisation"));
  P->state = 1;
  P->nonfinite = 0;
  if (P->nf) {
    // NaN or Inf in the exit waves propagate into S and D_p: count them
    unsigned long long h = 0;
    TRY(hip_check(launch_fill_zero(P->nf, 8, P->st), "non-finite check"));
    TRY(hip_check(launch_count_nonfinite(P->S, (int64_t)P->n_om * P->n_k, P->nf, P->st),
                  "non-finite check"));
    if (P->d.n_det > 0)
      TRY(hip_check(launch_count_nonfinite(P->Dp, (int64_t)P->d.n_det * P->d.n_probe * P->n_om,
                                           P->nf, P->st),
                    "non-finite check"));
    TRY(hip_check(hipMemcpyAsync(&h, P->nf, 8, hipMemcpyDeviceToHost, P->st), "non-finite check"));
    TRY(hip_check(hipStreamSynchronize(P->st), "non-finite check"));
    P->nonfinite = (int64_t)h;
    if (h > 0)
      return fail(TACAW_ERR_NONFINITE, std::to_string(h) +
                                           " non-finite values in S and D_p (NaN or Inf in the "
                                           "exit waves)");
  }
  return TACAW_OK;
}

int tacaw_detector_spectra(tacaw_plan_t P, const double* d_masks, int32_t n_det, double* d_D,
                           double* d_Dp) {
  g_err.clear();
  if (!P) return fail(TACAW_ERR_INVALID_ARG, "plan is NULL");
  if (P->state != 1) return fail(TACAW_ERR_STATE, "plan is not finalized");
  const double* masks = d_masks ? d_masks : P->masks;
  if (!d_masks && n_det != P->d.n_det)
    return fail(TACAW_ERR_INVALID_ARG, "n_det must equal the plan's when using the plan's masks");
  if (n_det < 0 || n_det > kMaxDet) return fail(TACAW_ERR_INVALID_ARG, "n_det must be in [0, 8]");
  if (n_det > 0 && !masks) return fail(TACAW_ERR_INVALID_ARG, "no masks");
  if (d_Dp && (d_masks || P->d.n_det == 0))
    return fail(TACAW_ERR_INVALID_ARG, "per-probe spectra need the plan's own masks");
  if (n_det > 0 && !d_D && !d_Dp) return fail(TACAW_ERR_INVALID_ARG, "no output");
  if (n_det > 0 && d_D) {
    TRY(hip_check(launch_fill_zero(d_D, (int64_t)n_det * P->n_om * 8, P->st), "zero D"));
    TRY(hip_check(launch_detector(P->S, masks, n_det, P->n_om, P->n_k, d_D, P->st), "detector"));
  }
  if (d_Dp)
    TRY(hip_check(hipMemcpyAsync(d_Dp, P->Dp, (size_t)P->d.n_det * P->d.n_probe * P->n_om * 8,
                                 hipMemcpyDeviceToDevice, P->st),
                  "per-probe copy"));
  return TACAW_OK;
}

}  // extern "C"

// Fixed device scratch of tacaw_backward_static: one copy per GPU, held until the
// process ends. Host code never passes `scratch` itself to a kernel (in host code
// it is only a stand-in for the symbol); it uses the per-device address below.
constexpr int64_t kStaticScratchBytes = TACAW_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's `scratch`, looked up once per device (the device
// must be current).
static int static_scratch(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return fail(TACAW_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(TACAW_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TACAW_OK;
}

// The adjoint, with its scratch (gmean [n_probes][n_k] double2, then the tile
// partials [n_tiles][2] double) either grown in the plan (fixed == nullptr) or
// taken from `fixed` of fixed_bytes (nothing allocated).
static int backward_impl(tacaw_plan_t P, const void* frames, int32_t probe0, int32_t n_probes,
                         int64_t pstride, int64_t fstride, const double* gS, const double* gD,
                         const double* gDp, void* grad, double* grad_wparam, void* fixed,
                         int64_t fixed_bytes) {
  if (!P) return fail(TACAW_ERR_INVALID_ARG, "plan is NULL");
  if (P->state != 1) return fail(TACAW_ERR_STATE, "plan is not finalized");
  if (!frames || !grad) return fail(TACAW_ERR_INVALID_ARG, "frames and grad must be given");
  if (((uintptr_t)frames) % P->esz != 0 || ((uintptr_t)grad) % P->esz != 0)
    return fail(TACAW_ERR_INVALID_ARG, "frames/grad not aligned to their element size");
  if (n_probes < 1 || probe0 < 0 || probe0 + (int64_t)n_probes > P->d.n_probe)
    return fail(TACAW_ERR_SHAPE, "probe range outside the plan");
  if (fstride < P->span)
    return fail(TACAW_ERR_INVALID_ARG, "frame_stride must cover a frame ((ny - 1) * row stride + nx)");
  if (n_probes > 1 && pstride < 1) return fail(TACAW_ERR_INVALID_ARG, "probe_stride must be >= 1");
  if (((int64_t)P->N2 * fstride + P->span) * P->esz > (int64_t)0x7FFFFFFFLL)
    return fail(TACAW_ERR_UNSUPPORTED, "frame_stride too large for 31-bit row-group offsets");
  if (P->H != P->L && 2 * P->H != P->L)
    return fail(TACAW_ERR_UNSUPPORTED, "backward supports hop = L or hop = L/2");
  if (bwd_tile_pixels(P->L) == 0)
    return fail(TACAW_ERR_UNSUPPORTED, "backward supports seg_len 64 ... 1024 (powers of two) and 200");
  if ((gD || gDp) && P->d.n_det == 0)
    return fail(TACAW_ERR_INVALID_ARG, "detector gradients need plan masks");
  if (bwd_pass1_size(P->L) != P->N1)
    return fail(TACAW_ERR_UNSUPPORTED, "the adjoint's DFT split differs from the plan's tables");
  const bool global = P->d.mean_mode == TACAW_MEAN_GLOBAL;
  const bool per_chunk = P->d.mean_mode == TACAW_MEAN_PER_SEGMENT;
  // the mean term comes from the forward pass's bin sums when the window's DFT
  // lives on bins 0, +-1 (those sums exist); otherwise a second pass applies it.
  // Per-chunk means (compact windows only) are applied inside the kernel.
  const int n_corr = ((global || per_chunk) && P->strategy == kRefSampled) ? P->n_corr : 0;
  const int Wb = bwd_tile_pixels(P->L);
  const int n_tiles = (P->n_k + Wb - 1) / Wb;
  const int64_t need = (int64_t)n_probes * P->n_k * 16 + (int64_t)n_tiles * 16;
  double* work = P->scratch;
  if (fixed) {
    if (need > fixed_bytes)
      return fail(TACAW_ERR_SHAPE, "the adjoint needs " + std::to_string(need) +
                                       " bytes of scratch, more than the fixed " +
                                       std::to_string(fixed_bytes) + " (16 n_probes n_k + 16 tiles)");
    work = (double*)fixed;
  } else if (need > P->scratch_bytes) {
    P->release((void**)&P->scratch);
    P->scratch_bytes = 0;
    TRY(P->alloc((void**)&P->scratch, need, "adjoint scratch"));
    P->scratch_bytes = need;
    work = P->scratch;
  }
  BwdArgs b{};
  b.in = frames;
  b.pstride = pstride;
  b.fstride = fstride;
  b.nx = P->d.nx;
  b.row_stride = P->rs;
  b.grad = grad;
  b.n_k = P->n_k;
  b.probe0 = probe0;
  b.n_probes = n_probes;
  b.n_probe_total = P->d.n_probe;
  b.n_seg = P->Ns;
  b.hop = P->H;
  b.n_det = P->d.n_det;
  b.n_om = P->n_om;
  b.roi_half = P->roi;
  b.mean_global = global ? 1 : 0;
  b.per_chunk = per_chunk ? 1 : 0;
  b.cmean = P->cmean;
  b.inv_nused = 1.0 / (double)P->n_used;
  b.n_used = P->n_used;
  b.win_t = P->win_t;
  b.dwin_t = P->d.window == TACAW_WIN_HANN_WIDTH ? P->dwin_t : nullptr;
  b.tw = P->tw;
  b.cref = P->cref;
  b.msum = P->msum;
  b.xs = P->xs;
  b.n_corr = n_corr;
  for (int i = 0; i < kMaxCorr; ++i) b.wbin[i] = P->wbin[i];
  b.gS = gS;
  b.gD = gD;
  b.gDp = gDp;
  b.masks = P->masks;
  b.kappa_S = kappa_S(P);
  b.kappa_p = kappa_probe(P);
  b.qfac = P->qfac;
  // (every scratch value the adjoint's kernels read is written earlier in the same call)
  b.gmean = (double2*)work;
  b.dwpart = work + (int64_t)n_probes * P->n_k * 2;
  TRY(hip_check(launch_bwd(P->L, P->d.in_dtype, b, n_tiles, P->st), "adjoint kernel"));
  if (global && n_corr == 0)
    TRY(hip_check(launch_bwd_mean_fix(b, P->d.in_dtype, P->st), "adjoint mean term"));
  if (grad_wparam && P->d.window == TACAW_WIN_HANN_WIDTH) {
    const std::vector<double> w = make_window(P->d.window, P->L, P->d.window_param);
    const std::vector<double> dw = make_window_dr(P->L, P->d.window_param);
    double swd = 0.0;
    for (int t = 0; t < P->L; ++t) swd += w[t] * dw[t];
    TRY(hip_check(launch_bwd_wparam(b.dwpart, n_tiles, swd / P->sumw2, grad_wparam, P->st),
                  "window-parameter gradient"));
  }
  return TACAW_OK;
}

extern "C" {

int tacaw_backward(tacaw_plan_t P, const void* frames, int32_t probe0, int32_t n_probes,
                   int64_t pstride, int64_t fstride, const double* gS, const double* gD,
                   const double* gDp, void* grad, double* grad_wparam) {
  g_err.clear();
  return backward_impl(P, frames, probe0, n_probes, pstride, fstride, gS, gD, gDp, grad,
                       grad_wparam, nullptr, 0);
}

int tacaw_backward_static(tacaw_plan_t P, const void* frames, int32_t probe0, int32_t n_probes,
                          int64_t pstride, int64_t fstride, const double* gS, const double* gD,
                          const double* gDp, void* grad, double* grad_wparam) {
  g_err.clear();
  if (!P) return fail(TACAW_ERR_INVALID_ARG, "plan is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(TACAW_ERR_HIP, "no current HIP device");
  }
  if (dev != P->device) return fail(TACAW_ERR_INVALID_ARG, "the plan's device must be current");
  void* fixed = nullptr;
  TRY(static_scratch(dev, &fixed));
  return backward_impl(P, frames, probe0, n_probes, pstride, fstride, gS, gD, gDp, grad,
                       grad_wparam, fixed, kStaticScratchBytes);
}

}  // extern "C"

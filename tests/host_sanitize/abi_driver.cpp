// Host-side driver of the C ABI for the AddressSanitizer / UndefinedBehaviorSanitizer
// build (tests/test_host_sanitizers.py). It runs every validation path that needs no
// GPU: descriptor checks, the plan's host preparation (windows, the window's DFT,
// the transform split and tables, mean strategy) up to the first device call, and
// the argument checks of every other entry point. On a machine without a GPU each
// tacaw_plan call stops at the device query and must release what it built.
// Exit status 0 when every call returned what is expected; the sanitizers report
// memory and undefined-behaviour errors themselves.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tacaw.h"

static int g_fail = 0;

static void expect(bool ok, const char* what, int rc) {
  if (!ok) {
    std::printf("FAIL %s: rc %d (%s)\n", what, rc, tacaw_last_error());
    ++g_fail;
  }
}

static tacaw_plan_desc base() {
  tacaw_plan_desc d;
  std::memset(&d, 0, sizeof d);
  d.n_probe = 2;
  d.ny = 8;
  d.nx = 8;
  d.n_frames = 256;
  d.seg_len = 128;
  d.hop = 64;
  d.window = TACAW_WIN_HANN;
  d.window_param = 1.0;
  d.mean_mode = TACAW_MEAN_GLOBAL;
  d.transform = TACAW_FFT_F32;
  d.in_dtype = TACAW_C64;
  d.probe_reduce = TACAW_PROBE_MEAN;
  d.dt_fs = 5.0;
  return d;
}

// a descriptor that must be refused by tacaw_plan_check (and by tacaw_plan)
static void refused(const tacaw_plan_desc& d, const char* what) {
  const int rc = tacaw_plan_check(&d);
  expect(rc != TACAW_OK && std::strlen(tacaw_last_error()) > 0, what, rc);
  tacaw_plan_t p = reinterpret_cast<tacaw_plan_t>(1);
  const int rc2 = tacaw_plan(&d, nullptr, &p);
  expect(rc2 == rc && p == nullptr, what, rc2);
}

// a valid descriptor: the check passes; the plan either builds (a GPU is present)
// or stops at the first device call with HIP or OOM. The plan itself refuses the
// per-chunk mean for windows whose DFT is not confined to bins 0 and +-1 (it
// builds the window before it can tell).
static void accepted(const tacaw_plan_desc& d, const char* what) {
  const int rc = tacaw_plan_check(&d);
  expect(rc == TACAW_OK, what, rc);
  tacaw_plan_t p = nullptr;
  const int rc2 = tacaw_plan(&d, nullptr, &p);
  const bool refused_window = rc2 == TACAW_ERR_UNSUPPORTED &&
                              d.mean_mode == TACAW_MEAN_PER_SEGMENT &&
                              d.window != TACAW_WIN_HANN && d.window != TACAW_WIN_RECT;
  expect(rc2 == TACAW_OK || rc2 == TACAW_ERR_HIP || rc2 == TACAW_ERR_OOM || refused_window, what,
         rc2);
  expect((rc2 == TACAW_OK) == (p != nullptr), what, rc2);
  if (p) {
    tacaw_plan_info info;
    expect(tacaw_plan_get_info(p, &info) == TACAW_OK, "info of a built plan", 0);
    tacaw_destroy(p);
  }
}

int main() {
  expect(std::strlen(tacaw_version()) > 0, "version", 0);
  expect(tacaw_last_error() != nullptr, "last_error", 0);

  // ---- descriptor checks, one bad field at a time ----
  expect(tacaw_plan_check(nullptr) == TACAW_ERR_INVALID_ARG, "NULL desc", 0);
  {
    tacaw_plan_t p = nullptr;
    tacaw_plan_desc d = base();
    expect(tacaw_plan(&d, nullptr, nullptr) == TACAW_ERR_INVALID_ARG, "NULL out", 0);
    expect(tacaw_plan(nullptr, nullptr, &p) == TACAW_ERR_INVALID_ARG && p == nullptr,
           "NULL desc plan", 0);
  }
  struct Bad {
    const char* what;
    void (*set)(tacaw_plan_desc&);
  };
  const Bad bad[] = {
      {"n_probe 0", [](tacaw_plan_desc& d) { d.n_probe = 0; }},
      {"ny 0", [](tacaw_plan_desc& d) { d.ny = 0; }},
      {"nx -3", [](tacaw_plan_desc& d) { d.nx = -3; }},
      {"grid 2^32", [](tacaw_plan_desc& d) { d.ny = 1 << 16; d.nx = 1 << 16; }},
      {"seg_len 96", [](tacaw_plan_desc& d) { d.seg_len = 96; }},
      {"seg_len 2048", [](tacaw_plan_desc& d) { d.seg_len = 2048; d.n_frames = 4096; }},
      {"seg_len 32", [](tacaw_plan_desc& d) { d.seg_len = 32; d.hop = 16; }},
      {"seg_len 200 with GEMM", [](tacaw_plan_desc& d) {
         d.seg_len = 200;
         d.hop = 100;
         d.n_frames = 400;
         d.transform = TACAW_GEMM_BF16X3;
       }},
      {"hop 0", [](tacaw_plan_desc& d) { d.hop = 0; }},
      {"hop > L", [](tacaw_plan_desc& d) { d.hop = 129; }},
      {"n_frames < L", [](tacaw_plan_desc& d) { d.n_frames = 127; }},
      {"window 9", [](tacaw_plan_desc& d) { d.window = 9; }},
      {"window -1", [](tacaw_plan_desc& d) { d.window = -1; }},
      {"custom without values", [](tacaw_plan_desc& d) { d.window = TACAW_WIN_CUSTOM; }},
      {"temperature NaN", [](tacaw_plan_desc& d) { d.temperature_K = std::nan(""); }},
      {"temperature < 0", [](tacaw_plan_desc& d) { d.temperature_K = -1.0; }},
      {"width-r 0", [](tacaw_plan_desc& d) {
         d.window = TACAW_WIN_HANN_WIDTH;
         d.window_param = 0.0;
       }},
      {"width-r 5", [](tacaw_plan_desc& d) {
         d.window = TACAW_WIN_HANN_WIDTH;
         d.window_param = 5.0;
       }},
      {"Tukey 1.5", [](tacaw_plan_desc& d) { d.window = TACAW_WIN_TUKEY; d.window_param = 1.5; }},
      {"Tukey NaN", [](tacaw_plan_desc& d) {
         d.window = TACAW_WIN_TUKEY;
         d.window_param = std::nan("");
       }},
      {"mean mode 7", [](tacaw_plan_desc& d) { d.mean_mode = 7; }},
      {"transform 3", [](tacaw_plan_desc& d) { d.transform = 3; }},
      {"GEMM at L 64", [](tacaw_plan_desc& d) {
         d.seg_len = 64;
         d.hop = 32;
         d.transform = TACAW_GEMM_BF16X3;
       }},
      {"per-chunk mean with fp16 GEMM", [](tacaw_plan_desc& d) {
         d.mean_mode = TACAW_MEAN_PER_SEGMENT;
         d.transform = TACAW_GEMM_F16X3;
       }},
      {"per-chunk mean, hop < L/4", [](tacaw_plan_desc& d) {
         d.mean_mode = TACAW_MEAN_PER_SEGMENT;
         d.hop = 16;
       }},
      {"per-chunk mean, 2^31 frames", [](tacaw_plan_desc& d) {
         d.mean_mode = TACAW_MEAN_PER_SEGMENT;
         d.n_frames = (int64_t)1 << 31;
       }},
      {"in_dtype 2", [](tacaw_plan_desc& d) { d.in_dtype = 2; }},
      {"probe_reduce 2", [](tacaw_plan_desc& d) { d.probe_reduce = 2; }},
      {"dt 0", [](tacaw_plan_desc& d) { d.dt_fs = 0.0; }},
      {"dt NaN", [](tacaw_plan_desc& d) { d.dt_fs = std::nan(""); }},
      {"n_det 9", [](tacaw_plan_desc& d) { d.n_det = 9; }},
      {"n_det without masks", [](tacaw_plan_desc& d) { d.n_det = 2; }},
      {"in flight > n_probe", [](tacaw_plan_desc& d) { d.max_probes_in_flight = 3; }},
      {"in flight < 0", [](tacaw_plan_desc& d) { d.max_probes_in_flight = -1; }},
      {"omega_half L/2", [](tacaw_plan_desc& d) { d.omega_half = 64; }},
      {"omega_half < 0", [](tacaw_plan_desc& d) { d.omega_half = -2; }},
      {"row stride < nx", [](tacaw_plan_desc& d) { d.k_row_stride = 7; }},
      {"ring = L", [](tacaw_plan_desc& d) { d.ring_frames = 128; }},
      {"ring not a multiple of L/2", [](tacaw_plan_desc& d) { d.ring_frames = 200; }},
      {"ring 2^30", [](tacaw_plan_desc& d) { d.ring_frames = (int64_t)1 << 30; }},
      {"ring with fp16 GEMM", [](tacaw_plan_desc& d) {
         d.ring_frames = 256;
         d.transform = TACAW_GEMM_F16X3;
       }},
      {"tiled without ring", [](tacaw_plan_desc& d) { d.flags = TACAW_FLAG_TILED_RING; }},
      {"tiled with hop != L/2", [](tacaw_plan_desc& d) {
         d.flags = TACAW_FLAG_TILED_RING;
         d.ring_frames = 256;
         d.hop = 32;
       }},
      {"accumulators beyond device memory", [](tacaw_plan_desc& d) {
         d.ny = 1 << 15;
         d.nx = 1 << 15;
         d.n_probe = 100000;
         d.seg_len = 1024;
         d.hop = 512;
         d.n_frames = 4096;
       }},
  };
  for (const Bad& b : bad) {
    tacaw_plan_desc d = base();
    b.set(d);
    refused(d, b.what);
  }
  {  // an all-zero custom window is refused by the plan (after the check)
    std::vector<double> zero(128, 0.0);
    tacaw_plan_desc d = base();
    d.window = TACAW_WIN_CUSTOM;
    d.h_window = zero.data();
    tacaw_plan_t p = nullptr;
    const int rc = tacaw_plan(&d, nullptr, &p);
    expect(rc == TACAW_ERR_INVALID_ARG && p == nullptr, "zero custom window", rc);
  }

  // ---- valid descriptors through the plan's host preparation ----
  const int lens[] = {64, 128, 200, 256, 512, 1024};
  const int windows[] = {TACAW_WIN_HANN, TACAW_WIN_RECT, TACAW_WIN_HANN_WIDTH, TACAW_WIN_TUKEY,
                         TACAW_WIN_CUSTOM};
  const int transforms[] = {TACAW_FFT_F32, TACAW_GEMM_BF16X3, TACAW_GEMM_F16X3};
  const int means[] = {TACAW_MEAN_GLOBAL, TACAW_MEAN_PER_SEGMENT, TACAW_MEAN_NONE};
  char what[160];
  for (int L : lens) {
    std::vector<double> bh(L);  // a four-term Blackman-Harris window (App. A), periodic
    for (int t = 0; t < L; ++t) {
      const double x = 2.0 * M_PI * t / L;
      bh[t] = 0.35875 - 0.48829 * std::cos(x) + 0.14128 * std::cos(2 * x) -
              0.01168 * std::cos(3 * x);
    }
    for (int win : windows) {
      for (int tr : transforms) {
        for (int mm : means) {
          for (int roi : {0, 5, L / 2 - 1}) {
            tacaw_plan_desc d = base();
            d.seg_len = L;
            d.hop = L / 2;
            d.n_frames = 3 * L + 17;
            d.window = win;
            d.window_param =
                win == TACAW_WIN_TUKEY ? 0.1 : (win == TACAW_WIN_HANN_WIDTH ? 0.5 : 1.0);
            d.h_window = win == TACAW_WIN_CUSTOM ? bh.data() : nullptr;
            d.transform = tr;
            d.mean_mode = mm;
            d.omega_half = roi;
            d.temperature_K = roi == 5 ? 300.0 : 0.0;
            d.in_dtype = roi == 0 ? TACAW_C64 : TACAW_C128;
            std::snprintf(what, sizeof what, "L %d window %d transform %d mean %d roi %d", L, win,
                          tr, mm, roi);
            const int rc = tacaw_plan_check(&d);
            if (rc == TACAW_OK) {
              accepted(d, what);
            } else {
              // the only refusals in this grid: GEMM at L 64 or 200, per-chunk mean with
              // fp16 GEMM; and the plan refuses per-chunk mean with non-compact windows
              expect(rc == TACAW_ERR_UNSUPPORTED, what, rc);
              refused(d, what);
            }
          }
        }
      }
    }
    // streaming options at this length
    tacaw_plan_desc d = base();
    d.seg_len = L;
    d.hop = L / 2;
    d.n_frames = 8 * L;
    d.max_probes_in_flight = 1;
    if (L % 2 == 0 && L != 200) {
      d.ring_frames = 4 * L;
      std::snprintf(what, sizeof what, "L %d deferred ring", L);
      accepted(d, what);
      d.flags = TACAW_FLAG_TILED_RING;
      std::snprintf(what, sizeof what, "L %d tiled ring", L);
      accepted(d, what);
    }
    d = base();
    d.seg_len = L;
    d.hop = L;
    d.n_frames = 2 * L;
    d.k_row_stride = 11;
    d.probe_reduce = TACAW_PROBE_SUM;
    d.flags = TACAW_FLAG_CHECK_FINITE | TACAW_FLAG_TIME_KERNELS;
    std::snprintf(what, sizeof what, "L %d k window, sum, finite check", L);
    accepted(d, what);
  }

  // ---- the other entry points reject a NULL plan before any device call ----
  double x = 0.0;
  void* dst = nullptr;
  int64_t a = 0, b = 0, c = 0;
  int32_t tp = 0;
  tacaw_plan_info info;
  expect(tacaw_push_frames(nullptr, &x, 0, 1, 1, 1, 1) == TACAW_ERR_INVALID_ARG, "push NULL", 0);
  expect(tacaw_ingest_frames(nullptr, 0, 1, 1, &dst, &a, &b) == TACAW_ERR_INVALID_ARG,
         "ingest NULL", 0);
  expect(tacaw_ingest_frames_tiled(nullptr, 0, 1, 1, &dst, &a, &b, &c, &tp) ==
             TACAW_ERR_INVALID_ARG,
         "ingest tiled NULL", 0);
  expect(tacaw_commit_frames(nullptr, 0, 1, 1) == TACAW_ERR_INVALID_ARG, "commit NULL", 0);
  expect(tacaw_finalize(nullptr, &x) == TACAW_ERR_INVALID_ARG, "finalize NULL", 0);
  expect(tacaw_detector_spectra(nullptr, nullptr, 0, &x, nullptr) == TACAW_ERR_INVALID_ARG,
         "detectors NULL", 0);
  expect(tacaw_backward(nullptr, &x, 0, 1, 1, 1, &x, nullptr, nullptr, &x, nullptr) ==
             TACAW_ERR_INVALID_ARG,
         "backward NULL", 0);
  expect(tacaw_backward_static(nullptr, &x, 0, 1, 1, 1, &x, nullptr, nullptr, &x, nullptr) ==
             TACAW_ERR_INVALID_ARG,
         "backward_static NULL", 0);
  expect(tacaw_reset(nullptr) == TACAW_ERR_INVALID_ARG, "reset NULL", 0);
  expect(tacaw_set_stream(nullptr, nullptr) == TACAW_ERR_INVALID_ARG, "set_stream NULL", 0);
  expect(tacaw_plan_get_info(nullptr, &info) == TACAW_ERR_INVALID_ARG, "info NULL", 0);
  unsigned char state[64] = {0};
  expect(tacaw_plan_export(nullptr, state, sizeof state, &a) == TACAW_ERR_INVALID_ARG,
         "export NULL", 0);
  expect(tacaw_plan_import(nullptr, state, sizeof state) == TACAW_ERR_INVALID_ARG, "import NULL",
         0);

  // ---- state merge (host only), on forged states with the exported layout ----
  {
    struct Head {  // format tag, fingerprint, size, probes, pixels, bins, detectors,
      uint64_t magic, fp;  // per-chunk flag, S defined, frames dropped
      int64_t total;
      int32_t np, nk, nom, ndet, pc, sdef;
      int64_t dropped;
    };
    const int np = 3, nb = 20;
    const int64_t bytes = (int64_t)sizeof(Head) + np * 8 + nb * 8;
    std::vector<unsigned char> sa((size_t)bytes), sb((size_t)bytes), so((size_t)bytes);
    auto fill = [&](std::vector<unsigned char>& v, int64_t c0, int64_t c1, int64_t c2, double x) {
      const Head h{0x31305354574154ull, 7, bytes, np, 4, 5, 1, 0, 1, 3};
      std::memcpy(v.data(), &h, sizeof h);
      const int64_t c[3] = {c0, c1, c2};
      std::memcpy(v.data() + sizeof h, c, sizeof c);
      for (int i = 0; i < nb; ++i) {
        const double d = x + i;
        std::memcpy(v.data() + sizeof h + np * 8 + i * 8, &d, 8);
      }
    };
    fill(sa, 9, 0, 0, 1.0);
    fill(sb, 0, 9, 9, 2.0);
    int rc = tacaw_state_merge(sa.data(), sb.data(), so.data(), bytes);
    expect(rc == TACAW_OK, "merge", rc);
    double last = 0.0;
    std::memcpy(&last, so.data() + bytes - 8, 8);
    expect(last == 1.0 + 19 + 2.0 + 19, "merge sum", 0);
    rc = tacaw_state_merge(sa.data(), sb.data(), sa.data(), bytes);
    expect(rc == TACAW_OK, "merge in place", rc);
    rc = tacaw_state_merge(sa.data(), sb.data(), so.data(), bytes);  // now overlapping
    expect(rc == TACAW_ERR_INVALID_ARG, "merge overlap", rc);
    rc = tacaw_state_merge(sb.data(), sb.data(), so.data(), bytes - 8);
    expect(rc == TACAW_ERR_SHAPE, "merge size", rc);
    rc = tacaw_state_merge(sb.data(), sb.data(), so.data(), 16);
    expect(rc == TACAW_ERR_SHAPE, "merge short", rc);
    rc = tacaw_state_merge(nullptr, sb.data(), so.data(), bytes);
    expect(rc == TACAW_ERR_INVALID_ARG, "merge NULL", rc);
  }
  tacaw_destroy(nullptr);

  // ---- producer and read probes: argument checks ----
  {
    tacaw_synth_desc s;
    std::memset(&s, 0, sizeof s);
    float tab[4] = {0, 0, 0, 0};
    double tan_tab[4] = {0, 0, 0, 0};
    alignas(8) unsigned char buf[64];
    expect(tacaw_synth_frames(nullptr, buf, 0, 1, 0, 1, 1, 1, 0, 1, nullptr) ==
               TACAW_ERR_INVALID_ARG,
           "synth NULL desc", 0);
    s.ny = 0;
    s.nx = 4;
    expect(tacaw_synth_frames(&s, buf, 0, 1, 0, 1, 1, 1, 0, 1, nullptr) == TACAW_ERR_SHAPE,
           "synth ny 0", 0);
    s.ny = 4;
    s.n_terms = 17;
    expect(tacaw_synth_frames(&s, buf, 0, 1, 0, 1, 1, 1, 0, 1, nullptr) == TACAW_ERR_INVALID_ARG,
           "synth 17 terms", 0);
    s.n_terms = 2;
    s.n_lines = 3;
    expect(tacaw_synth_frames(&s, buf, 0, 1, 0, 1, 1, 1, 0, 1, nullptr) == TACAW_ERR_INVALID_ARG,
           "synth without tables", 0);
    s.d_cos = tab;
    s.d_sin = tab;
    s.d_tan = tan_tab;
    s.noise_sigma = 1e-5;
    expect(tacaw_synth_frames(&s, buf, 0, 1, 0, 1, 1, 1, 0, 1, nullptr) == TACAW_ERR_INVALID_ARG,
           "synth noise without normals", 0);
    s.noise_sigma = 0.0;
    expect(tacaw_synth_frames(&s, buf, -1, 1, 0, 1, 1, 1, 0, 16, nullptr) == TACAW_ERR_SHAPE,
           "synth probe0 < 0", 0);
    expect(tacaw_synth_frames(&s, buf, 0, 1, (int64_t)1 << 32, 1, 1, 1, 0, 16, nullptr) ==
               TACAW_ERR_SHAPE,
           "synth frames beyond 2^32", 0);
    expect(tacaw_synth_frames(&s, buf, 0, 1, 0, 1, 1, 0, 0, 16, nullptr) == TACAW_ERR_INVALID_ARG,
           "synth frame stride 0", 0);
    expect(tacaw_synth_frames(&s, buf + 4, 0, 1, 0, 1, 1, 1, 0, 16, nullptr) ==
               TACAW_ERR_INVALID_ARG,
           "synth misaligned", 0);
    expect(tacaw_synth_frames(&s, buf, 0, 1, 0, 0, 1, 1, 0, 16, nullptr) == TACAW_OK,
           "synth zero frames", 0);
  }
  {
    uint64_t sum = 0;
    alignas(16) unsigned char buf[64];
    expect(tacaw_read_probe(nullptr, 16, nullptr, &sum) == TACAW_ERR_INVALID_ARG, "read NULL", 0);
    expect(tacaw_read_probe(buf, 15, nullptr, &sum) == TACAW_ERR_INVALID_ARG, "read 15 bytes", 0);
    expect(tacaw_read_probe_columns(buf, 2, 128, 48, nullptr, &sum) == TACAW_ERR_INVALID_ARG,
           "columns seg 48", 0);
    expect(tacaw_read_probe_columns(buf, 2, 100, 64, nullptr, &sum) == TACAW_ERR_INVALID_ARG,
           "columns ragged row", 0);
  }

  std::printf("%s: %d failed expectations\n", g_fail ? "FAIL" : "OK", g_fail);
  return g_fail ? 1 : 0;
}

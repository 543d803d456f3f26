// Host side of librx.so: the C ABI of include/rx.h, filter design in FP64,
// workspace management and launch sequencing (single buffers, batches and
// hipGraph replay of batches).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <unistd.h>
#include <tuple>
#include <vector>

#include "../../include/rx.h"
#include "rx_shared.h"

namespace {

thread_local char g_err[256] = "";

int fail_hip(hipError_t e, const char *what) {
  snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
  return RX_E_HIP;
}

bool is_kk(int fmt) { return fmt == RX_KK_QPSK || fmt == RX_KK_16QAM; }
int bps_of(int fmt) { return fmt == RX_PAM2 ? 1 : fmt == RX_PAM4 ? 2 : fmt == RX_PAM8 ? 3 : fmt == RX_KK_QPSK ? 2 : 4; }
int axis_levels(int fmt) { return fmt == RX_PAM2 ? 2 : fmt == RX_PAM4 ? 4 : fmt == RX_PAM8 ? 8 : fmt == RX_KK_QPSK ? 2 : 4; }

// ---- FP64 designs, rounded once to FP32 ----------------------------------
// Root-raised-cosine taps at `sps` samples/symbol, closed form including the
// limits at t = 0 and |t| = 1/(4 beta), unit energy.
std::vector<double> design_rrc(int k, double sps, double beta) {
  std::vector<double> h(k);
  double e = 0.0;
  for (int i = 0; i < k; i++) {
    const double t = (i - 0.5 * (k - 1)) / sps;
    double v;
    if (std::fabs(t) < 1e-12) {
      v = 1.0 - beta + 4.0 * beta / M_PI;
    } else if (beta > 0 && std::fabs(std::fabs(t) - 0.25 / beta) < 1e-12) {
      const double a = M_PI / (4.0 * beta);
      v = beta / std::sqrt(2.0) * ((1.0 + 2.0 / M_PI) * std::sin(a) + (1.0 - 2.0 / M_PI) * std::cos(a));
    } else {
      const double q = 4.0 * beta * t;
      v = (std::sin(M_PI * t * (1.0 - beta)) + q * std::cos(M_PI * t * (1.0 + beta))) / (M_PI * t * (1.0 - q * q));
    }
    h[i] = v;
    e += v * v;
  }
  for (auto &v : h) v /= std::sqrt(e);
  return h;
}

// Hilbert FIR h(m), |m| <= V/2: (2/(pi m)) Blackman(m) for odd m, else 0;
// returned for m = 1..V/2 (odd symmetric).  Its N-point DFT is -j S[k] with
// S[k] = 2 sum_{m>0} h(m) sin(2 pi k m / N).
std::vector<float> design_hilbert_spectrum(int ntaps, int log2n, double scale = 1.0) {
  const int v = ntaps - 1, half = v / 2, n = 1 << log2n;
  std::vector<double> h(half + 1, 0.0);
  for (int m = 1; m <= half; m += 2) {
    const double w = 0.42 + 0.5 * std::cos(2.0 * M_PI * m / v) + 0.08 * std::cos(4.0 * M_PI * m / v);
    h[m] = 2.0 / (M_PI * m) * w;
  }
  std::vector<double> sn(n);
  for (int i = 0; i < n; i++) sn[i] = std::sin(2.0 * M_PI * i / n);
  std::vector<float> s(n);
  for (int k = 0; k < n; k++) {
    double acc = 0.0;
    for (int m = 1; m <= half; m += 2) acc += h[m] * sn[(int)(((int64_t)k * m) % n)];
    s[k] = (float)(scale * 2.0 * acc / n);
  }
  return s;
}

std::vector<float2> design_twiddles(int log2n) {
  const int n = 1 << log2n;
  std::vector<float2> t(n);
  for (int k = 0; k < n; k++) t[k] = make_float2((float)std::cos(2.0 * M_PI * k / n), (float)-std::sin(2.0 * M_PI * k / n));
  return t;
}

struct Alloc {
  std::vector<void *> ptrs;
  template <class T>
  T *get(size_t count) {
    void *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<T *>(p);
  }
  ~Alloc() {
    for (void *p : ptrs) hipFree(p);
  }
};

struct GraphCache {
  std::vector<uint64_t> key;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;   // library stream used only for capture (the null stream cannot be captured)
};

}  // namespace

struct rx_ctx {
  rx_format fmt;
  rx_params p;
  uint64_t uid = 0;       // unique over the process: never reused by a later handle
  uint64_t version = 0;   // bumped whenever the device job or the stage list can change
  int wall_khz = 100000;  // device wall-clock rate
  int kk = 0, sps = 2, bps = 1, log2n = 14;
  RxTune tune = {14, 8, 8, 2048};   // launch shapes
  hipStream_t stream = nullptr;
  RxJob hj{};
  RxJob *dj = nullptr;
  RxScalars *dsc = nullptr;
  Alloc mem;
  int64_t last_n = 0;
  GraphCache graph;
  float *mlp = nullptr;   // learned-equaliser parameters (device), allocated with the handle
  void *scratch = nullptr;   // this device's static gradient partials (rx_mlp_grad_static)
  bool mlp_ready = false;
  uint8_t *hin = nullptr, *hbits = nullptr;   // host-ingest staging (device), allocated on first use
  // contiguous stream (RX_STREAM): the input of a buffer after the first is
  // the stream's previous hold + look samples (tail) followed by the buffer
  int64_t stream_pos = 0;      // stream samples received so far
  bool acquired = false;       // the stream's first buffer has been processed
  int64_t tail_n = 0;          // hold + look
  uint8_t *sx = nullptr, *stail = nullptr;
  // stage timing (RX_PROFILE): events recorded around every stage launch
  struct Pending { int stage; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double stage_ms[ST_COUNT] = {0};
  uint64_t stage_n[ST_COUNT] = {0};
  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
  }
  ~rx_ctx() {
    for (auto &p : pending) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
    for (auto e : pool) hipEventDestroy(e);
  }
};

extern "C" {

int rx_params_default(rx_format fmt, rx_params *p) {
  if (!p || fmt < RX_PAM2 || fmt > RX_KK_16QAM) return RX_E_INVALID;
  std::memset(p, 0, sizeof(*p));
  const bool kk = is_kk(fmt);
  p->struct_size = sizeof(rx_params);
  p->mf_taps = kk ? 65 : 33;
  p->ffe_taps = kk ? 21 : 15;
  p->prefix_symbols = 4096;
  p->hilbert_taps = 4097;
  p->fft_log2 = 0;
  p->precision = RX_FP32;
  p->equalizer = RX_EQ_LMS;
  p->rolloff = 0.1;
  p->mu = 1e-3;
  p->mu_cma = 1e-3;
  p->carrier_hz = kk ? 0.55e9 : 0.0;
  p->seed = 0;
  p->max_samples = (uint64_t)1 << 22;
  p->stream = nullptr;
  p->flags = 0;
  p->deadline_s = 0.0;
  p->ref_bits = nullptr;
  p->ref_period = 0;
  p->blocks_bc = 0;
  p->ffe_gpw = 0;
  p->dec_syms = 0;
  p->front = RX_FRONT_OS;
  return RX_OK;
}

const char *rx_strerror(int code) {
  switch (code) {
    case RX_OK: return "ok";
    case RX_E_INVALID: return "invalid argument";
    case RX_E_UNSUPPORTED: return "unsupported configuration";
    case RX_E_NOMEM: return "device allocation failed";
    case RX_E_HIP: return g_err[0] ? g_err : "HIP error";
    case RX_E_STATE: return "call-order violation";
    case RX_W_FALLBACK: return "warning: LMS fallback used";
    default: return "unknown status";
  }
}

// Hilbert spectrum and FFT twiddles depend only on (N, Hilbert taps): one
// copy per device serves every handle, so a batch of many buffers reads one
// L2-resident set of tables.  They are kept until the process ends.
struct SharedTables {
  float *hspec;
  float2 *twid;
};
static const SharedTables *shared_tables(int log2n, int htaps) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int>, SharedTables> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, log2n, htaps);
  auto it = cache.find(key);
  if (it != cache.end()) return &it->second;
  const int n = 1 << log2n;
  // the front end transforms log2 v, not ln sqrt v = (ln 2 / 2) log2 v, and
  // takes the phase in revolutions: the spectrum carries both factors
  const double rev = 0.5 * std::log(2.0) / (2.0 * M_PI);
  std::vector<float> hs = design_hilbert_spectrum(htaps, log2n, rev);
  std::vector<float2> tw = design_twiddles(log2n);
  // the 2^14-point front end runs its transforms as 16 x 1024: behind the
  // N-point twiddles the 1024-point ones, and behind the spectrum a copy in
  // the order its 1024-point transforms hand their outputs over (entry
  // 1024 k1 + 64 i + l is bin k = k1 + 16 (l + 64 i))
  const std::vector<float2> tw1k = design_twiddles(10);
  tw.insert(tw.end(), tw1k.begin(), tw1k.end());
  hs.resize(2 * (size_t)n, 0.0f);
  if (log2n == 14)
    for (int k1 = 0; k1 < 16; k1++)
      for (int i = 0; i < 16; i++)
        for (int l = 0; l < 64; l++) hs[n + 1024 * k1 + 64 * i + l] = hs[k1 + 16 * (l + 64 * i)];
  // then the same 2N entries negated, for the other sideband (sgn = -1)
  hs.resize(4 * (size_t)n);
  for (size_t k = 0; k < 2 * (size_t)n; k++) hs[2 * (size_t)n + k] = -hs[k];
  SharedTables t{nullptr, nullptr};
  if (hipMalloc((void **)&t.hspec, hs.size() * sizeof(float)) != hipSuccess) return nullptr;
  if (hipMalloc((void **)&t.twid, tw.size() * sizeof(float2)) != hipSuccess ||
      hipMemcpy(t.hspec, hs.data(), hs.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.twid, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(t.hspec);
    if (t.twid) hipFree(t.twid);
    return nullptr;
  }
  return &(cache[key] = t);
}

// Tables of the frequency-domain front ends, one copy per (device, roll-off,
// chain): hspec holds S[k] = sgn(k) / 1024 (block-circular Hilbert: -j S,
// zero at DC and N/2) and then the static equaliser's response over the 1024
// bins, divided by 1024 (the matched RRC, 203 taps at 4 sps for KK, 503 at
// 2 sps for PAM, centred, so real); twid holds the 1024-point twiddles and
// then the 512-point ones.
static const SharedTables *fd_tables(double rolloff, bool kk) {
  static std::mutex mu;
  static std::map<std::tuple<int, double, bool>, SharedTables> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, rolloff, kk);
  auto it = cache.find(key);
  if (it != cache.end()) return &it->second;
  constexpr int N = 1 << RX_KK_FD_LOG2;
  const int EQ = kk ? 203 : 503;   // the paper's static equaliser lengths (KK, PAM)
  std::vector<float> hs(2 * N);
  for (int k = 0; k < N; k++) hs[k] = (k == 0 || k == N / 2) ? 0.0f : (k < N / 2 ? 1.0f : -1.0f) / N;
  const std::vector<double> heq = design_rrc(EQ, kk ? 4.0 : 2.0, rolloff);
  for (int k = 0; k < N; k++) {
    double acc = 0.0;
    for (int i = 0; i < EQ; i++) acc += heq[i] * std::cos(2.0 * M_PI * (double)(((int64_t)k * (i - EQ / 2)) % N + N) / N);
    hs[N + k] = (float)(acc / N);
  }
  std::vector<float2> tw = design_twiddles(RX_KK_FD_LOG2), tw2 = design_twiddles(RX_KK_FD_LOG2 - 1);
  tw.insert(tw.end(), tw2.begin(), tw2.end());
  SharedTables t{nullptr, nullptr};
  if (hipMalloc((void **)&t.hspec, hs.size() * sizeof(float)) != hipSuccess) return nullptr;
  if (hipMalloc((void **)&t.twid, tw.size() * sizeof(float2)) != hipSuccess ||
      hipMemcpy(t.hspec, hs.data(), hs.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.twid, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(t.hspec);
    if (t.twid) hipFree(t.twid);
    return nullptr;
  }
  return &(cache[key] = t);
}

// ---- launch-shape tuner ----------------------------------------------------
// Each tunable shape (overlap-save FFT size, DD-LMS chunk steps, precision-form
// FFE groups per wavefront, decision symbols per workgroup) is chosen by
// timing its own stage on the device: a batch of 16 buffers of 2^22
// pseudo-random codes (the work does not depend on the values; the batch
// fills the chip as a streaming batch does, at the real buffer size) runs
// through the chain with HIP events around every stage, one candidate at a
// time with the others held at the current choice; the best of three runs
// counts, and a candidate must beat the incumbent by more than 3 %.  Choices
// are kept per (GPU architecture, chain, precision, FFE length) for the
// process and in a JSON file ($RX_TUNE_CACHE, else
// $HOME/.cache/paper_2010_14333_amd/autotune.json; an empty RX_TUNE_CACHE
// keeps them in memory only), so later processes on the same GPU model skip
// the timing.
static const RxTune kDefaultTune = {14, 8, 8, 2048};

static std::string tune_cache_path() {
  const char *e = std::getenv("RX_TUNE_CACHE");
  if (e) return std::string(e);
  const char *home = std::getenv("HOME");
  if (!home || !*home) return std::string();
  return std::string(home) + "/.cache/paper_2010_14333_amd/autotune.json";
}

// The cache file: {"key": {"fft_log2": a, "blocks_bc": b, "ffe_gpw": c, "dec_syms": d}, ...}
static std::map<std::string, RxTune> tune_file_read(const std::string &path) {
  std::map<std::string, RxTune> out;
  FILE *f = path.empty() ? nullptr : std::fopen(path.c_str(), "rb");
  if (!f) return out;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  size_t pos = 0;
  while (true) {
    const size_t k0 = text.find('"', pos);
    if (k0 == std::string::npos) break;
    const size_t k1 = text.find('"', k0 + 1);
    const size_t b0 = text.find('{', k1 == std::string::npos ? k0 : k1);
    const size_t b1 = text.find('}', b0 == std::string::npos ? k0 : b0);
    if (k1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
    const std::string key = text.substr(k0 + 1, k1 - k0 - 1), body = text.substr(b0 + 1, b1 - b0 - 1);
    RxTune t = kDefaultTune;
    int found = 0;
    const char *names[4] = {"\"fft_log2\"", "\"blocks_bc\"", "\"ffe_gpw\"", "\"dec_syms\""};
    int32_t *fields[4] = {&t.fft_log2, &t.blocks_bc, &t.ffe_gpw, &t.dec_syms};
    for (int i = 0; i < 4; i++) {
      const size_t q = body.find(names[i]);
      const size_t c = q == std::string::npos ? q : body.find(':', q);
      if (c == std::string::npos) continue;
      *fields[i] = (int32_t)std::strtol(body.c_str() + c + 1, nullptr, 10);
      found++;
    }
    if (found == 4) out[key] = t;
    pos = b1 + 1;
  }
  return out;
}

static void tune_file_write(const std::string &path, const std::map<std::string, RxTune> &m) {
  if (path.empty()) return;
  for (size_t i = 1; i < path.size(); i++)   // the directories (mkdir -p)
    if (path[i] == '/') mkdir(path.substr(0, i).c_str(), 0755);
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  FILE *f = std::fopen(tmp.c_str(), "wb");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (const auto &kv : m) {
    const RxTune &t = kv.second;
    std::fprintf(f, "  \"%s\": {\"fft_log2\": %d, \"blocks_bc\": %d, \"ffe_gpw\": %d, \"dec_syms\": %d}%s\n",
                 kv.first.c_str(), t.fft_log2, t.blocks_bc, t.ffe_gpw, t.dec_syms, ++i < m.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  if (std::fclose(f) == 0) std::rename(tmp.c_str(), path.c_str());
  else std::remove(tmp.c_str());
}

static int create_tuned(rx_format fmt, double baud, double fs, const rx_params *pin, const RxTune &t, rx_handle *out);

// Per-launch time (ms) of `stage` for the chain with tune t, best of three.
static float time_stage(rx_format fmt, double baud, double fs, const rx_params &p, const RxTune &t, int stage,
                        const void *dbuf, uint8_t *dbits, size_t n, size_t nbits) {
  constexpr int NB = 16;
  rx_params q = p;
  q.max_samples = n;
  q.flags = 0;
  q.stream = nullptr;
  q.ref_bits = nullptr;
  std::vector<rx_handle> hs;
  for (int i = 0; i < NB; i++) {
    rx_params qi = q;
    if (i == 0) qi.flags = RX_PROFILE;
    rx_handle h = nullptr;
    if (create_tuned(fmt, baud, fs, &qi, t, &h) != RX_OK) break;
    hs.push_back(h);
  }
  float best = -1.0f;
  if ((int)hs.size() == NB) {
    std::vector<const void *> bufs(NB, dbuf);
    std::vector<size_t> ns(NB, n);
    std::vector<void *> outs(NB);
    for (int i = 0; i < NB; i++) outs[i] = dbits + i * nbits;
    rx_process_batch(hs.data(), bufs.data(), ns.data(), outs.data(), NB, 0);   // warm-up
    for (int r = 0; r < 3; r++) {
      rx_stage_times(hs[0], nullptr, nullptr, 0);
      rx_process_batch(hs.data(), bufs.data(), ns.data(), outs.data(), NB, 0);
      double ms[RX_NSTAGES];
      uint64_t cnt[RX_NSTAGES];
      if (rx_stage_times(hs[0], ms, cnt, RX_NSTAGES) >= 0 && cnt[stage] > 0) {
        const float v = (float)(ms[stage] / cnt[stage]);
        if (best < 0.0f || v < best) best = v;
      }
    }
  }
  for (rx_handle h : hs) rx_destroy(h);
  return best;
}

static RxTune tune_shapes(rx_format fmt, double baud, double fs, const rx_params &p) {
  static std::mutex mu;
  static std::map<std::string, RxTune> known;
  static bool file_read = false;
  const bool kk = is_kk(fmt);
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return kDefaultTune;
  const std::string key = std::string(prop.gcnArchName) + "|" + (kk ? "kk" : "pam") + "|" +
                          std::to_string(p.precision) + "|" + std::to_string(p.ffe_taps) +
                          (p.front == RX_FRONT_FD ? "|fd" : "");
  std::lock_guard<std::mutex> lock(mu);
  const std::string path = tune_cache_path();
  if (!file_read) {
    known = tune_file_read(path);
    file_read = true;
  }
  auto it = known.find(key);
  if (it != known.end()) return it->second;

  RxTune t = kDefaultTune;
  constexpr int NB = 16;
  const size_t n = (size_t)1 << 22, nbits = n / 2;   // >= n / sps * bps / 8 for every format
  std::vector<uint8_t> host(3 * n / 2);
  uint64_t x = 0x2545F4914F6CDD1Dull;
  for (auto &b : host) {
    x ^= x << 13; x ^= x >> 7; x ^= x << 17;
    b = (uint8_t)(x >> 24);
  }
  void *dbuf = nullptr;
  uint8_t *dbits = nullptr;
  if (hipMalloc(&dbuf, host.size()) == hipSuccess && hipMalloc((void **)&dbits, NB * nbits) == hipSuccess &&
      hipMemcpy(dbuf, host.data(), host.size(), hipMemcpyHostToDevice) == hipSuccess) {
    struct Knob { int32_t RxTune::*field; std::vector<int32_t> cand; int stage; bool used; };
    const Knob knobs[] = {
        {&RxTune::fft_log2, {14, 13}, RX_ST_KK_FRONT, kk && p.front != RX_FRONT_FD},
        {&RxTune::blocks_bc, {8, 4, 16}, RX_ST_BLOCKS, !(kk && p.precision != RX_FP32)},
        {&RxTune::ffe_gpw, {8, 4, 16}, RX_ST_BLOCKS, kk && p.precision != RX_FP32},
        {&RxTune::dec_syms, {2048, 1024, 4096}, RX_ST_DECIDE, true},
    };
    for (const Knob &k : knobs) {
      if (!k.used) continue;
      float best_ms = -1.0f;
      int32_t best = t.*(k.field);
      for (int32_t c : k.cand) {   // the incumbent first
        RxTune tc = t;
        tc.*(k.field) = c;
        const float ms = time_stage(fmt, baud, fs, p, tc, k.stage, dbuf, dbits, n, nbits);
        if (ms > 0.0f && (best_ms < 0.0f || ms < 0.97f * best_ms)) {
          best_ms = ms;
          best = c;
        }
      }
      t.*(k.field) = best;
    }
  }
  if (dbuf) hipFree(dbuf);
  if (dbits) hipFree(dbits);
  known[key] = t;
  tune_file_write(path, known);
  return t;
}

int rx_create(rx_format fmt, double baud, double fs, const rx_params *pin, rx_handle *out) {
  return create_tuned(fmt, baud, fs, pin, RxTune{0, 0, 0, 0}, out);
}

// rx_create with launch shapes: fields of `forced` that are non-zero are used
// as they are (the tuner's candidates), the others come from the params or,
// where those leave them to the library, from the tuner.
static int create_tuned(rx_format fmt, double baud, double fs, const rx_params *pin, const RxTune &forced,
                        rx_handle *out) {
  if (!out) return RX_E_INVALID;
  *out = nullptr;
  rx_params p;
  if (rx_params_default(fmt, &p) != RX_OK) return RX_E_INVALID;
  if (pin) {
    if (pin->struct_size != sizeof(rx_params)) return RX_E_INVALID;
    p = *pin;
  }
  const bool kk = is_kk(fmt);
  const double sps = fs / baud;
  if (!(baud > 0) || !(fs > 0) || std::fabs(sps - (kk ? 4.0 : 2.0)) > 1e-9) return RX_E_UNSUPPORTED;
  if (p.mf_taps < 1 || p.mf_taps % 2 == 0 || p.mf_taps > (kk ? 65 : 33)) return RX_E_INVALID;
  if (p.ffe_taps != 15 && p.ffe_taps != 21 && !(kk && p.ffe_taps == 4)) return RX_E_UNSUPPORTED;
  if ((p.flags & RX_DD_PHASE) && !kk) return RX_E_UNSUPPORTED;
  if (p.prefix_symbols < 2048 || p.prefix_symbols > RX_PREFIX_MAX) return RX_E_INVALID;
  if (kk && (p.hilbert_taps < 3 || p.hilbert_taps > 4097 || p.hilbert_taps % 2 == 0)) return RX_E_INVALID;
  if (p.fft_log2 != 0 && p.fft_log2 != 13 && p.fft_log2 != 14) return RX_E_INVALID;
  if ((p.blocks_bc != 0 && p.blocks_bc != 4 && p.blocks_bc != 8 && p.blocks_bc != 16) ||
      (p.ffe_gpw != 0 && p.ffe_gpw != 4 && p.ffe_gpw != 8 && p.ffe_gpw != 16) ||
      (p.dec_syms != 0 && p.dec_syms != 1024 && p.dec_syms != 2048 && p.dec_syms != 4096))
    return RX_E_INVALID;
  if (!(p.rolloff > 0 && p.rolloff <= 1) || !(p.mu > 0) || !(p.mu_cma > 0)) return RX_E_INVALID;
  if (p.precision != RX_FP32 && p.precision != RX_BF16 && p.precision != RX_FP16) return RX_E_INVALID;
  if (p.precision != RX_FP32 && (!kk || p.ffe_taps != 21)) return RX_E_UNSUPPORTED;
  if (p.equalizer != RX_EQ_LMS && p.equalizer != RX_EQ_MLP) return RX_E_INVALID;
  if (p.equalizer == RX_EQ_MLP && kk) return RX_E_UNSUPPORTED;
  if (kk && !(std::fabs(p.carrier_hz) < fs / 2)) return RX_E_INVALID;
  if (p.max_samples < 65536 || p.max_samples > ((uint64_t)1 << 26) || p.max_samples % 1024) return RX_E_INVALID;
  if (!(p.deadline_s >= 0.0) || (reinterpret_cast<uintptr_t>(p.ref_bits) & 3)) return RX_E_INVALID;
  const bool stream = (p.flags & RX_STREAM) != 0;
  if (stream && p.ref_bits) return RX_E_UNSUPPORTED;   // a stream's reference outgrows any one buffer
  if (p.front != RX_FRONT_OS && p.front != RX_FRONT_FD) return RX_E_INVALID;
  const bool fd = p.front == RX_FRONT_FD;
  if (fd && (p.precision != RX_FP32 || stream || p.equalizer != RX_EQ_LMS)) return RX_E_UNSUPPORTED;
  int wall_khz = 0;
  {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess || wall_khz <= 0) return fail_hip(e != hipSuccess ? e : hipErrorInvalidValue, "wall clock rate");
  }

  static std::atomic<uint64_t> next_uid{1};
  rx_ctx *h = new rx_ctx();
  h->uid = next_uid.fetch_add(1);
  h->wall_khz = wall_khz;
  h->fmt = fmt;
  h->p = p;
  h->kk = kk;
  h->sps = kk ? 4 : 2;
  h->bps = bps_of(fmt);
  {
    // the launch shapes: forced (tuning), else given, else tuned
    RxTune t{forced.fft_log2 ? forced.fft_log2 : p.fft_log2, forced.blocks_bc ? forced.blocks_bc : p.blocks_bc,
             forced.ffe_gpw ? forced.ffe_gpw : p.ffe_gpw, forced.dec_syms ? forced.dec_syms : p.dec_syms};
    if (!kk && !t.fft_log2) t.fft_log2 = 14;   // no overlap-save transform in the PAM chain
    if (fd) t.fft_log2 = RX_KK_FD_LOG2;         // the paper's 1024-point blocks
    if (!(kk && p.precision != RX_FP32) && !t.ffe_gpw) t.ffe_gpw = 8;
    if (!t.fft_log2 || !t.blocks_bc || !t.ffe_gpw || !t.dec_syms) {
      const RxTune tuned = tune_shapes(fmt, baud, fs, p);
      if (!t.fft_log2) t.fft_log2 = tuned.fft_log2;
      if (!t.blocks_bc) t.blocks_bc = tuned.blocks_bc;
      if (!t.ffe_gpw) t.ffe_gpw = tuned.ffe_gpw;
      if (!t.dec_syms) t.dec_syms = tuned.dec_syms;
    }
    h->tune = t;
  }
  h->log2n = h->tune.fft_log2;
  h->stream = static_cast<hipStream_t>(p.stream);
  // a stream buffer after the first is processed with its prepended tail
  const int64_t L = (int64_t)p.max_samples + (stream ? (kk ? 2 * RX_KK_HOLD : 2 * RX_PAM_HOLD) : 0);
  Alloc &A = h->mem;
  RxJob &J = h->hj;
  J.fmt = fmt;
  J.kk = kk;
  J.bps = h->bps;
  J.m_axis = axis_levels(fmt);
  J.mf_taps = p.mf_taps;
  J.ffe_taps = p.ffe_taps;
  J.prefix = p.prefix_symbols;
  J.precision = p.precision;
  J.fft_log2 = h->log2n;
  // the frequency-domain front end writes one set of sums per 512-sample
  // block, which is what the prefix stage's count of ceil(ceil(n / hop) / 2)
  // gives with hop 256
  J.hop = fd ? 256 : rx_kk_hop(h->log2n);
  J.blk = kk ? 128 : 256;
  J.equalizer = p.equalizer;
  J.mu = (float)p.mu;
  J.mu_cma = (float)p.mu_cma;
  J.r2 = fmt == RX_KK_16QAM ? 1.32f : 1.0f;
  const int m = J.m_axis;
  J.ea2_sqrt = (float)std::sqrt((m * m - 1) / 3.0 * (kk ? 2.0 : 1.0));
  J.r = kk ? p.carrier_hz / fs : 0.0;
  J.sgn = p.carrier_hz >= 0 ? 1.0f : -1.0f;
  J.debug = (p.flags & RX_DEBUG_KEEP) ? 1 : 0;
  J.seed = p.seed;
  J.stream = stream ? 1 : 0;
  J.dd_phase = (p.flags & RX_DD_PHASE) ? 1 : 0;
  J.hold = kk ? RX_KK_HOLD : RX_PAM_HOLD;
  J.look = J.hold;
  J.ref_period = p.ref_period;
  h->tail_n = stream ? (int64_t)J.hold + J.look : 0;
  J.deadline_ticks = p.deadline_s * 1e3 * wall_khz;
  J.ticks_per_sample = 1e3 * wall_khz / fs;

  // matched filter: KK taps centred in 65 slots (zero padded)
  std::vector<double> hm = design_rrc(p.mf_taps, h->sps, p.rolloff);
  const int slots = kk ? 65 : 33;
  std::vector<float> hf(slots, 0.0f);
  std::vector<double> hd(slots, 0.0);
  for (int i = 0; i < p.mf_taps; i++) {
    hd[(slots - p.mf_taps) / 2 + i] = hm[i];
    hf[(slots - p.mf_taps) / 2 + i] = (float)hm[i];
  }
  // precision form: the filter is the narrow-rounded taps (the carrier term
  // removed after it uses the same filter)
  for (int i = 0; i < slots; i++) {
    if (p.precision == RX_BF16) hf[i] = (float)(__bf16)hf[i];
    else if (p.precision == RX_FP16) hf[i] = (float)(_Float16)hf[i];
  }
  if (fd) std::fill(hf.begin(), hf.end(), 0.0f);   // no carrier term: the FD output is carrier-free
  float *dmf = A.get<float>(slots);
  bool ok = dmf != nullptr;
  if (ok) ok = hipMemcpy(dmf, hf.data(), slots * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
  J.mf = dmf;
  if (kk && ok) {
    // interior value of MF(exp(-j 2 pi r n)) at n = 2m, divided by exp(-j 2 pi r 2m)
    std::complex<double> c0 = 0.0;
    for (int i = 0; i < 65; i++) c0 += (double)hf[i] * std::exp(std::complex<double>(0.0, -2.0 * M_PI * J.r * (32 - i)));
    J.c0 = make_float2((float)c0.real(), (float)c0.imag());
    const SharedTables *t = fd ? fd_tables(p.rolloff, true) : shared_tables(h->log2n, p.hilbert_taps);
    ok = t != nullptr;
    if (ok) {
      // the overlap-save front end's spectrum copy for this sideband
      J.hspec = t->hspec + (!fd && J.sgn < 0.0f ? 2 * ((size_t)1 << h->log2n) : 0);
      J.twid = t->twid;
    }
    const int64_t nd = L / 2;
    const int hop = J.hop;
    J.z = A.get<float2>(nd);
    J.part = A.get<double2>(3 * (((L + hop - 1) / hop + 1) / 2 + 1));
    J.soft = A.get<float2>(L / 4);
    J.s4 = A.get<float2>(L / 4 / 128);
    J.theta = A.get<float>(L / 4 / 128);
    J.field = J.debug ? A.get<float2>(L) : nullptr;
    J.udbg = J.debug ? A.get<float2>(nd) : nullptr;
    ok = ok && J.z && J.part && J.soft && J.s4 && J.theta && (!J.debug || (J.field && J.udbg));
    if (fd) {
      J.phi = A.get<float>(L);
      J.fdpart = A.get<double2>(L / 1024 + 1);
      ok = ok && J.phi && J.fdpart;
    }
  } else if (ok) {
    J.y = A.get<float>(L);
    J.xr = A.get<float>(L);
    J.upart = A.get<uint32_t>(L / 16384 + 1);
    J.part2 = A.get<double>(L / 1024 + 1);   // per 4096-sample tile, or per 1024-sample FD block pair
    J.gard = A.get<float2>(L / 512);
    J.delta = A.get<float>(2 * (L / 512));
    J.soft = A.get<float2>(L / 2);
    ok = J.y && J.xr && J.upart && J.part2 && J.gard && J.delta && J.soft;
    if (ok && fd) {
      const SharedTables *t = fd_tables(p.rolloff, false);
      ok = t != nullptr;
      if (ok) {
        J.hspec = t->hspec;
        J.twid = t->twid;
      }
    }
  }
  if (ok && !kk) {
    h->mlp = A.get<float>(rx_mlp_params());
    ok = h->mlp != nullptr;
    if (ok) {
      const int se = rx_mlp_scratch_resolve(&h->scratch);
      if (se) {
        delete h;
        return fail_hip((hipError_t)se, "hipGetSymbolAddress (static gradient partials)");
      }
    }
  }
  // reference bits of every symbol a buffer of this handle can hold, unless
  // the caller supplies its own stream of them
  const int64_t nsym_max = L / (kk ? 4 : 2);
  const int64_t ref_words = (nsym_max * J.bps + 31) / 32;
  uint32_t *refw = nullptr;
  if (ok && !p.ref_bits) {
    refw = A.get<uint32_t>(ref_words);
    ok = refw != nullptr;
  }
  J.refw = p.ref_bits ? static_cast<const uint32_t *>(p.ref_bits) : refw;
  J.ref_ext = p.ref_bits ? 1 : 0;
  h->dsc = ok ? A.get<RxScalars>(1) : nullptr;
  h->dj = ok && h->dsc ? A.get<RxJob>(1) : nullptr;
  if (!h->dj) {
    delete h;
    return RX_E_NOMEM;
  }
  if (stream) {
    h->sx = A.get<uint8_t>(L / 2 * 3);
    h->stail = A.get<uint8_t>(h->tail_n / 2 * 3);
    if (!h->sx || !h->stail) {
      delete h;
      return RX_E_NOMEM;
    }
  }
  J.sc = h->dsc;
  RxScalars zero{};
  if (hipMemcpy(h->dsc, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->dj, &J, sizeof(J), hipMemcpyHostToDevice) != hipSuccess) {
    delete h;
    return fail_hip(hipGetLastError(), "rx_create upload");
  }
  if (refw) rx_launch_ref_fill(refw, ref_words, J.seed, J.bps, nsym_max, J.ref_period, nullptr);
  if (hipStreamSynchronize(nullptr) != hipSuccess) {
    delete h;
    return fail_hip(hipGetLastError(), "rx_create reference bits");
  }
  *out = h;
  return RX_OK;
}

static int check_n(rx_handle h, size_t n) {
  if (n == 0 || n % 1024 || n > h->p.max_samples) return RX_E_INVALID;
  const int64_t nsym = (int64_t)n / h->sps;
  if (h->hj.stream && h->acquired) return RX_OK;   // any whole number of granules continues a stream
  const int64_t held = h->hj.stream ? h->tail_n / h->sps : 0;   // a stream's first buffer also fills the tail
  if (nsym < h->p.prefix_symbols + 2 * RX_GUARD + 128 + held) return RX_E_INVALID;
  return RX_OK;
}

// Symbols a call emits: all of an independent buffer; a stream's first
// buffer holds its last `hold` samples back, later ones emit exactly their
// own length (the decisions of the previous buffer's held samples first).
static int64_t emitted_symbols(rx_handle h, size_t n) {
  if (!h->hj.stream) return (int64_t)n / h->sps;
  return h->acquired ? (int64_t)n / h->sps : ((int64_t)n - h->hj.hold) / h->sps;
}

// A stream buffer's input: the first one as it is; a later one after the
// stream's tail, assembled in the handle's staging area.  Returns the
// pointer and length to process and the launch's s0 (see RxLaunch).
static hipError_t stream_input(rx_handle h, const void *buf, size_t n, hipStream_t s, const void **in, int64_t *nx,
                               int64_t *s0) {
  if (!h->hj.stream || !h->acquired) {
    *in = buf;
    *nx = (int64_t)n;
    *s0 = -1;
    return hipSuccess;
  }
  const size_t tb = (size_t)h->tail_n / 2 * 3;
  hipError_t e = hipMemcpyAsync(h->sx, h->stail, tb, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h->sx + tb, buf, n / 2 * 3, hipMemcpyDeviceToDevice, s);
  *in = h->sx;
  *nx = h->tail_n + (int64_t)n;
  *s0 = h->stream_pos - h->tail_n;
  return e;
}

// After a stream buffer: its input's last hold + look samples become the tail.
static hipError_t stream_advance(rx_handle h, const void *in, int64_t nx, size_t n, hipStream_t s) {
  if (!h->hj.stream) return hipSuccess;
  const size_t tb = (size_t)h->tail_n / 2 * 3;
  const hipError_t e = hipMemcpyAsync(h->stail, static_cast<const uint8_t *>(in) + (size_t)(nx - h->tail_n) / 2 * 3, tb,
                                      hipMemcpyDeviceToDevice, s);
  h->stream_pos += (int64_t)n;
  h->acquired = true;
  return e;
}

static const int KK_STAGES[] = {ST_KK_FRONT, ST_PREFIX, ST_BLOCKS, ST_KK_VV, ST_DECIDE, ST_KK_DEBUG};
static const int PAM_STAGES[] = {ST_PAM_SUM, ST_PAM_MF, ST_PAM_GAVG, ST_PAM_UNWRAP, ST_PAM_FARROW,
                                 ST_PREFIX, ST_BLOCKS, ST_DECIDE};
static const int PAM_MLP_STAGES[] = {ST_PAM_SUM, ST_PAM_MF, ST_PAM_GAVG, ST_PAM_UNWRAP, ST_PAM_FARROW,
                                     ST_PREFIX, ST_MLP_INFER, ST_MLP_JUDGE, ST_BLOCKS, ST_DECIDE};
// a stream buffer after the first: the acquisition (means, gain, delay,
// rotation, prefix taps, network judgement) is the stream's
static const int KK_CONT_STAGES[] = {ST_KK_FRONT, ST_BLOCKS, ST_KK_VV, ST_DECIDE, ST_KK_DEBUG};
static const int PAM_CONT_STAGES[] = {ST_PAM_MF, ST_PAM_GAVG, ST_PAM_UNWRAP, ST_PAM_FARROW, ST_BLOCKS, ST_DECIDE};
static const int PAM_MLP_CONT_STAGES[] = {ST_PAM_MF, ST_PAM_GAVG, ST_PAM_UNWRAP, ST_PAM_FARROW, ST_MLP_INFER,
                                          ST_BLOCKS, ST_DECIDE};

static bool uses_mlp(const rx_ctx *h) { return h->p.equalizer == RX_EQ_MLP && h->mlp_ready; }

// Launch the chains of one batch: jobs grouped by (chain, FFT size, taps),
// each group one launch per stage.  With RX_PROFILE on the first handle
// (and not under graph capture) every stage is bracketed by events.
// ns[i]: samples to process (a stream buffer's with its tail); s0[i]: see RxLaunch.
static int enqueue(rx_handle const *hs, const void *const *bufs, const int64_t *ns, const int64_t *s0,
                   void *const *bits, int count, hipStream_t s, bool capturing) {
  bool done[RX_MAXB] = {false};
  rx_ctx *prof = (!capturing && (hs[0]->p.flags & RX_PROFILE)) ? hs[0] : nullptr;
  for (int i = 0; i < count; i++) {
    if (done[i]) continue;
    RxLaunch L{};
    int64_t maxn = 0;
    const rx_ctx *a = hs[i];
    const bool cont = s0[i] >= 0;
    for (int j = i; j < count; j++) {
      const rx_ctx *b = hs[j];
      if (done[j] || b->kk != a->kk || b->log2n != a->log2n || b->p.ffe_taps != a->p.ffe_taps ||
          b->tune.blocks_bc != a->tune.blocks_bc || b->tune.ffe_gpw != a->tune.ffe_gpw ||
          b->tune.dec_syms != a->tune.dec_syms ||
          b->p.precision != a->p.precision || uses_mlp(b) != uses_mlp(a) || (s0[j] >= 0) != cont)
        continue;
      done[j] = true;
      L.job[L.count] = b->dj;
      L.in[L.count] = static_cast<const uint8_t *>(bufs[j]);
      L.bits[L.count] = static_cast<uint8_t *>(bits[j]);
      L.n[L.count] = ns[j];
      L.s0[L.count] = s0[j];
      L.count++;
      if (ns[j] > maxn) maxn = ns[j];
    }
    const int *st;
    int nst;
    if (cont) {
      st = a->kk ? KK_CONT_STAGES : (uses_mlp(a) ? PAM_MLP_CONT_STAGES : PAM_CONT_STAGES);
      nst = a->kk ? (a->hj.debug ? 5 : 4) : (uses_mlp(a) ? 7 : 6);
    } else {
      st = a->kk ? KK_STAGES : (uses_mlp(a) ? PAM_MLP_STAGES : PAM_STAGES);
      nst = a->kk ? (a->hj.debug ? 6 : 5) : (uses_mlp(a) ? 10 : 8);
    }
    for (int k = 0; k < nst; k++) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (prof) {
        e0 = prof->event();
        hipEventRecord(e0, s);
      }
      if (st[k] == ST_KK_FRONT || st[k] == ST_KK_DEBUG || st[k] == ST_KK_VV)
        rx_launch_kk_stage(st[k], L, maxn, a->log2n, a->p.precision, s);
      else if (st[k] >= ST_PAM_SUM && st[k] <= ST_PAM_FARROW)
        rx_launch_pam_stage(st[k], L, maxn, a->log2n, s);
      else if (st[k] == ST_MLP_INFER || st[k] == ST_MLP_JUDGE)
        rx_launch_mlp_stage(st[k], L, maxn, s);
      else
        rx_launch_eq_stage(st[k], L, maxn, a->kk, a->p.ffe_taps, a->p.precision, a->tune, s);
      if (prof) {
        e1 = prof->event();
        hipEventRecord(e1, s);
        prof->pending.push_back({st[k], e0, e1});
      }
    }
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? RX_OK : fail_hip(e, "kernel launch");
}

static bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3) == 0; }

int rx_process(rx_handle h, const void *dev_buffer, size_t n_samples, void *dev_bits, size_t *n_bits_out) {
  if (!h || !dev_buffer || !dev_bits || !aligned4(dev_buffer) || !aligned4(dev_bits)) return RX_E_INVALID;
  int rc = check_n(h, n_samples);
  if (rc) return rc;
  const int64_t nemit = emitted_symbols(h, n_samples);
  const void *in = nullptr;
  int64_t nx = 0, s0 = -1;
  hipError_t e = stream_input(h, dev_buffer, n_samples, h->stream, &in, &nx, &s0);
  if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync (stream input)");
  rc = enqueue(&h, &in, &nx, &s0, &dev_bits, 1, h->stream, false);
  if (rc) return rc;
  e = stream_advance(h, in, nx, n_samples, h->stream);
  if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync (stream tail)");
  h->last_n = nx;
  if (n_bits_out) *n_bits_out = (size_t)(nemit * h->bps);
  return (h->p.equalizer == RX_EQ_MLP && !h->mlp_ready) ? RX_W_FALLBACK : RX_OK;
}

int rx_tuning(rx_handle h, int32_t *shapes) {
  if (!h || !shapes) return RX_E_INVALID;
  shapes[0] = h->tune.fft_log2;
  shapes[1] = h->tune.blocks_bc;
  shapes[2] = h->tune.ffe_gpw;
  shapes[3] = h->tune.dec_syms;
  return RX_OK;
}

int rx_stream_reset(rx_handle h) {
  if (!h) return RX_E_INVALID;
  if (!h->hj.stream) return RX_E_STATE;
  const hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  h->stream_pos = 0;
  h->acquired = false;
  return RX_OK;
}

int rx_process_batch(const rx_handle *hs, const void *const *bufs, const size_t *ns, void *const *bits, int count,
                     int graph) {
  if (!hs || !bufs || !ns || !bits || count < 1 || count > RX_MAXB) return RX_E_INVALID;
  for (int i = 0; i < count; i++) {
    if (!hs[i] || !bufs[i] || !bits[i] || !aligned4(bufs[i]) || !aligned4(bits[i])) return RX_E_INVALID;
    if (hs[i]->stream != hs[0]->stream) return RX_E_INVALID;
    for (int j = 0; j < i; j++)
      if (hs[j] == hs[i]) return RX_E_INVALID;
    int rc = check_n(hs[i], ns[i]);
    if (rc) return rc;
  }
  hipStream_t s = hs[0]->stream;
  int rc = RX_OK;
  bool any_stream = false;
  for (int i = 0; i < count; i++) any_stream |= hs[i]->hj.stream != 0;
  if (graph && any_stream) return RX_E_UNSUPPORTED;   // a stream's launch arguments change every call
  const void *in[RX_MAXB];
  int64_t nx[RX_MAXB], s0[RX_MAXB];
  for (int i = 0; i < count; i++) {
    const hipError_t e = stream_input(hs[i], bufs[i], ns[i], s, &in[i], &nx[i], &s0[i]);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync (stream input)");
  }
  if (!graph) {
    rc = enqueue(hs, in, nx, s0, bits, count, s, false);
    for (int i = 0; i < count && rc == RX_OK; i++) {
      const hipError_t e = stream_advance(hs[i], in[i], nx[i], ns[i], s);
      if (e != hipSuccess) rc = fail_hip(e, "hipMemcpyAsync (stream tail)");
    }
  } else {
    GraphCache &gc = hs[0]->graph;
    // a graph replays the stage list and job pointers of the handles it was
    // captured with: keyed by each handle's process-unique id and version
    // (bumped whenever its job or its stage list can change), not by its
    // address, which a later handle may reuse
    std::vector<uint64_t> key;
    for (int i = 0; i < count; i++) {
      key.push_back(hs[i]->uid);
      key.push_back(hs[i]->version);
      key.push_back(reinterpret_cast<uintptr_t>(bufs[i]));
      key.push_back(reinterpret_cast<uintptr_t>(bits[i]));
      key.push_back((uint64_t)ns[i]);
    }
    if (!gc.exec || gc.key != key) {
      if (gc.exec) {
        hipGraphExecDestroy(gc.exec);
        gc.exec = nullptr;
      }
      hipGraph_t g = nullptr;
      hipError_t e = hipSuccess;
      if (!gc.capture) {
        e = hipStreamCreateWithFlags(&gc.capture, hipStreamNonBlocking);
        if (e != hipSuccess) return fail_hip(e, "hipStreamCreateWithFlags");
      }
      e = hipStreamBeginCapture(gc.capture, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return fail_hip(e, "hipStreamBeginCapture");
      rc = enqueue(hs, in, nx, s0, bits, count, gc.capture, true);
      e = hipStreamEndCapture(gc.capture, &g);
      if (rc) {
        if (g) hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) {
        gc.exec = nullptr;
        return fail_hip(e, "hipGraphInstantiate");
      }
      gc.key = key;
    }
    hipError_t e = hipGraphLaunch(gc.exec, s);
    if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
  }
  if (rc == RX_OK)
    for (int i = 0; i < count; i++) hs[i]->last_n = nx[i];
  return rc;
}

int rx_process_batch_host(const rx_handle *hs, const void *const *host_buffers, const size_t *ns,
                          void *const *host_bits, int count, int graph) {
  if (!hs || !host_buffers || !ns || !host_bits || count < 1 || count > RX_MAXB) return RX_E_INVALID;
  const void *dbufs[RX_MAXB];
  void *dbits[RX_MAXB];
  for (int i = 0; i < count; i++) {
    rx_ctx *h = hs[i];
    if (!h || !host_buffers[i] || !host_bits[i]) return RX_E_INVALID;
    if (h->stream != hs[0]->stream) return RX_E_INVALID;
    for (int j = 0; j < i; j++)
      if (hs[j] == h) return RX_E_INVALID;
    const int rc = check_n(h, ns[i]);
    if (rc) return rc;
    if (!h->hin) {
      h->hin = h->mem.get<uint8_t>(h->p.max_samples / 2 * 3);
      h->hbits = h->mem.get<uint8_t>(h->p.max_samples / h->sps * h->bps / 8);
      if (!h->hin || !h->hbits) {
        h->hin = h->hbits = nullptr;
        return RX_E_NOMEM;
      }
    }
    dbufs[i] = h->hin;
    dbits[i] = h->hbits;
  }
  hipStream_t s = hs[0]->stream;
  size_t nbytes[RX_MAXB];
  for (int i = 0; i < count; i++) nbytes[i] = (size_t)(emitted_symbols(hs[i], ns[i]) * hs[i]->bps / 8);
  for (int i = 0; i < count; i++) {
    const hipError_t e = hipMemcpyAsync(hs[i]->hin, host_buffers[i], ns[i] / 2 * 3, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync (buffer in)");
  }
  const int rc = rx_process_batch(hs, dbufs, ns, dbits, count, graph);
  if (rc) return rc;
  for (int i = 0; i < count; i++) {
    const size_t nb = nbytes[i];
    const hipError_t e = hipMemcpyAsync(host_bits[i], hs[i]->hbits, nb, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync (bits out)");
  }
  return RX_OK;
}

int rx_sync(rx_handle h) {
  if (!h) return RX_E_INVALID;
  const hipError_t e = hipStreamSynchronize(h->stream);
  return e == hipSuccess ? RX_OK : fail_hip(e, "hipStreamSynchronize");
}

int rx_errors(rx_handle h, rx_stats *out) {
  if (!h || !out) return RX_E_INVALID;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  unsigned long long st[7];
  e = hipMemcpy(st, h->dsc->stats, sizeof(st), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "hipMemcpy stats");
  out->buffers = st[0];
  out->symbols = st[1];
  out->bits = st[2];
  out->bit_errors = st[3];
  out->symbol_errors = st[4];
  out->fallbacks = st[5];
  out->late_buffers = st[6];
  return RX_OK;
}

int rx_latencies(rx_handle h, double *us, size_t max, size_t *count) {
  if (!h || (!us && max)) return RX_E_INVALID;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  unsigned long long c = 0;
  e = hipMemcpy(&c, &h->dsc->lat_count, sizeof(c), hipMemcpyDeviceToHost);
  std::vector<unsigned int> ring(RX_LAT_RING);
  if (e == hipSuccess) e = hipMemcpy(ring.data(), h->dsc->lat, sizeof(unsigned int) * RX_LAT_RING, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "hipMemcpy latencies");
  const size_t kept = (size_t)(c < RX_LAT_RING ? c : RX_LAT_RING);
  const size_t nout = kept < max ? kept : max;
  const double us_per_tick = 1e3 / h->wall_khz;
  for (size_t i = 0; i < nout; i++) {   // the most recent nout, oldest first
    const unsigned long long idx = c - nout + i;
    us[i] = ring[idx % RX_LAT_RING] * us_per_tick;
  }
  if (count) *count = nout;
  return RX_OK;
}

int rx_errors_reset(rx_handle h) {
  if (!h) return RX_E_INVALID;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  unsigned long long z[7] = {0, 0, 0, 0, 0, 0, 0};
  e = hipMemcpy(h->dsc->stats, z, sizeof(z), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(&h->dsc->lat_count, z, sizeof(z[0]), hipMemcpyHostToDevice);
  return e == hipSuccess ? RX_OK : fail_hip(e, "hipMemcpy stats");
}

int rx_debug_fetch(rx_handle h, int stage, void *dst, size_t bytes) {
  if (!h || !dst) return RX_E_INVALID;
  if (h->last_n == 0) return RX_E_STATE;
  const int64_t n = h->last_n, nsym = n / h->sps;
  const RxJob &J = h->hj;
  const void *src = nullptr;
  size_t need = 0;
  std::vector<double> scal;
  RxScalars sc;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  switch (stage) {
    case RX_STAGE_FIELD:
      if (!h->kk) return RX_E_INVALID;
      if (!J.field) return RX_E_STATE;
      src = J.field; need = n * sizeof(float2); break;
    case RX_STAGE_MF:
      if (h->kk && !J.udbg) return RX_E_STATE;
      src = h->kk ? (const void *)J.udbg : (const void *)J.y;
      need = h->kk ? (n / 2) * sizeof(float2) : n * sizeof(float); break;
    case RX_STAGE_XR:
      if (h->kk) return RX_E_INVALID;
      src = J.xr; need = n * sizeof(float); break;
    case RX_STAGE_TIMING:
      if (h->kk) return RX_E_INVALID;
      src = J.delta; need = (n / 512) * sizeof(float); break;
    case RX_STAGE_SOFT:
      if (h->kk && !J.debug) return RX_E_STATE;
      src = J.soft; need = nsym * (h->kk ? sizeof(float2) : sizeof(float)); break;   // PAM: real
    case RX_STAGE_TAPS:
      src = reinterpret_cast<const char *>(h->dsc) + offsetof(RxScalars, w0);
      need = h->p.ffe_taps * sizeof(float2); break;
    case RX_STAGE_PHASE:
      if (!h->kk) return RX_E_INVALID;
      src = J.theta; need = (nsym / 128) * sizeof(float); break;
    case RX_STAGE_SCALARS: {
      if (bytes != 8 * sizeof(double)) return RX_E_INVALID;
      e = hipMemcpy(&sc, h->dsc, sizeof(sc), hipMemcpyDeviceToHost);
      if (e != hipSuccess) return fail_hip(e, "hipMemcpy scalars");
      double v[8] = {sc.mean_re, sc.mean_im, sc.agc, sc.theta0, (double)sc.lag, (double)sc.rot, (double)sc.fallback, 0.0};
      std::memcpy(dst, v, sizeof(v));
      return RX_OK;
    }
    default: return RX_E_INVALID;
  }
  if (bytes != need) return RX_E_INVALID;
  e = hipMemcpy(dst, src, need, hipMemcpyDeviceToHost);
  return e == hipSuccess ? RX_OK : fail_hip(e, "hipMemcpy debug");
}


// ---- learned equaliser ----------------------------------------------------
static int upload_job(rx_handle h) {
  h->version++;   // cached graphs of this handle are stale from here on
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemcpy(h->dj, &h->hj, sizeof(RxJob), hipMemcpyHostToDevice);
  return e == hipSuccess ? RX_OK : fail_hip(e, "job upload");
}

int rx_train_cfg_default(rx_train_cfg *c) {
  if (!c) return RX_E_INVALID;
  std::memset(c, 0, sizeof(*c));
  c->struct_size = sizeof(rx_train_cfg);
  c->epochs = 2;
  c->batch = 1024;
  c->max_steps = 0;
  c->lr = 1e-3;
  c->beta1 = 0.9;
  c->beta2 = 0.999;
  c->eps = 1e-8;
  c->init_seed = 1;
  c->init = nullptr;
  return RX_OK;
}

int rx_mlp_param_count(void) { return rx_mlp_params(); }

int rx_set_mlp(rx_handle h, const float *host) {
  if (!h || !host) return RX_E_INVALID;
  if (!h->mlp) return RX_E_UNSUPPORTED;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemcpy(h->mlp, host, rx_mlp_params() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail_hip(e, "rx_set_mlp");
  h->mlp_ready = true;
  h->hj.mlp = h->p.equalizer == RX_EQ_MLP ? h->mlp : nullptr;
  return upload_job(h);
}

int rx_get_mlp(rx_handle h, float *host) {
  if (!h || !host) return RX_E_INVALID;
  if (!h->mlp) return RX_E_UNSUPPORTED;
  if (!h->mlp_ready) return RX_E_STATE;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemcpy(host, h->mlp, rx_mlp_params() * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? RX_OK : fail_hip(e, "rx_get_mlp");
}

static uint64_t mix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Kaiming-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero biases.
static std::vector<float> mlp_init(uint64_t seed) {
  const int np = rx_mlp_params();
  std::vector<float> w(np, 0.0f);
  auto fill = [&](int off, int count, int fan_in) {
    const double b = std::sqrt(6.0 / fan_in);
    for (int i = 0; i < count; i++) {
      const double u = (double)(mix64(seed, (uint64_t)(off + i)) >> 11) * (1.0 / 9007199254740992.0);
      w[off + i] = (float)((2.0 * u - 1.0) * b);
    }
  };
  fill(0, 64 * 31, 31);
  fill(64 * 31 + 64, 64 * 64, 64);
  fill(64 * 31 + 64 + 64 * 64 + 64, 64, 64);
  return w;
}

static int64_t gcd64(int64_t a, int64_t b) { return b ? gcd64(b, a % b) : a; }

#define RX_TRAIN_INFLIGHT 256

int rx_mlp_order_multiplier(int64_t ntrain) {
  int64_t m = 1000003;
  while (gcd64(m, ntrain) != 1) m += 2;
  return (int)m;
}

int rx_train_mlp_data(rx_handle h, const float *dev_x, const float *dev_t, size_t ntrain, const rx_train_cfg *cin,
                      double *final_loss) {
  if (!h || !dev_x || !dev_t || ntrain == 0) return RX_E_INVALID;
  if (!h->mlp) return RX_E_UNSUPPORTED;
  rx_train_cfg c;
  rx_train_cfg_default(&c);
  if (cin) {
    if (cin->struct_size != sizeof(rx_train_cfg)) return RX_E_INVALID;
    c = *cin;
  }
  if (c.batch < 1 || c.batch > 65536 || c.epochs < 1 || !(c.lr > 0)) return RX_E_INVALID;
  const int np = rx_mlp_params();
  std::vector<float> w0 = c.init ? std::vector<float>(c.init, c.init + np) : mlp_init(c.init_seed);
  const int nwg = (c.batch + 63) / 64;
  float *m = nullptr, *v = nullptr, *part = nullptr;
  double *loss = nullptr;
  hipError_t e = hipMalloc(&m, np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&v, np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&part, (size_t)nwg * np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&loss, nwg * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(h->mlp, w0.data(), np * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m, 0, np * sizeof(float));
  if (e == hipSuccess) e = hipMemset(v, 0, np * sizeof(float));
  int64_t steps = (int64_t)c.epochs * ((int64_t)ntrain / c.batch);
  if (steps < 1) steps = 1;
  if (c.max_steps > 0 && c.max_steps < steps) steps = c.max_steps;
  const int64_t mult = rx_mlp_order_multiplier((int64_t)ntrain);
  for (int64_t t = 0; t < steps && e == hipSuccess; t++) {
    const double c1 = 1.0 - std::pow(c.beta1, (double)(t + 1)), c2 = 1.0 - std::pow(c.beta2, (double)(t + 1));
    rx_mlp_step(dev_x, dev_t, (int64_t)ntrain, t * c.batch, c.batch, mult, h->mlp, m, v, part, loss, nullptr, 1,
                (float)c.lr, (float)c.beta1, (float)c.beta2, (float)c.eps, (float)c1, (float)c2, h->stream);
    e = hipGetLastError();
    // at most RX_TRAIN_INFLIGHT steps (two launches each) queued ahead of the
    // device: an unbounded queue of ~32k launches holds per-launch state in
    // the runtime and in any tool that intercepts launches
    if (e == hipSuccess && (t + 1) % RX_TRAIN_INFLIGHT == 0) e = hipStreamSynchronize(h->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess && final_loss) {
    std::vector<double> lp(nwg);
    e = hipMemcpy(lp.data(), loss, nwg * sizeof(double), hipMemcpyDeviceToHost);
    double acc = 0.0;
    for (double x : lp) acc += x;
    *final_loss = acc / c.batch;
  }
  hipFree(m);
  hipFree(v);
  hipFree(part);
  hipFree(loss);
  if (e != hipSuccess) return fail_hip(e, "rx_train_mlp_data");
  h->mlp_ready = true;
  h->hj.mlp = h->p.equalizer == RX_EQ_MLP ? h->mlp : nullptr;
  return upload_job(h);
}

int rx_train_mlp(rx_handle h, const void *const *dev_buffers, const size_t *n_samples, const uint64_t *seeds,
                 int count, const rx_train_cfg *c, double *final_loss) {
  if (!h || !dev_buffers || !n_samples || !seeds || count < 1) return RX_E_INVALID;
  if (h->kk || !h->mlp) return RX_E_UNSUPPORTED;
  int64_t rows = 0;
  for (int i = 0; i < count; i++) {
    int rc = check_n(h, n_samples[i]);
    if (rc) return rc;
    rows += (int64_t)n_samples[i] / 2 - 2 * RX_GUARD;
  }
  float *X = nullptr, *T = nullptr;
  hipError_t e = hipMalloc(&X, (size_t)rows * 32 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&T, (size_t)rows * sizeof(float));
  if (e != hipSuccess) {
    hipFree(X);
    return RX_E_NOMEM;
  }
  const uint64_t seed0 = h->hj.seed;
  const int32_t ext0 = h->hj.ref_ext;
  const float *mlp0 = h->hj.mlp;
  h->hj.mlp = nullptr;   // training buffers run the plain front end and prefix
  h->hj.ref_ext = 0;     // their known symbols come from their own seeds
  int rc = RX_OK;
  int64_t row0 = 0;
  for (int i = 0; i < count && rc == RX_OK; i++) {
    h->hj.seed = seeds[i];
    rc = upload_job(h);
    if (rc) break;
    RxLaunch L{};
    L.job[0] = h->dj;
    L.in[0] = static_cast<const uint8_t *>(dev_buffers[i]);
    L.n[0] = (int64_t)n_samples[i];
    L.count = 1;
    L.s0[0] = -1;   // an independent buffer
    for (int st = ST_PAM_SUM; st <= ST_PAM_FARROW; st++) rx_launch_pam_stage(st, L, L.n[0], h->log2n, h->stream);
    rx_launch_eq_stage(ST_PREFIX, L, L.n[0], 0, h->p.ffe_taps, 0, h->tune, h->stream);
    rx_mlp_windows(L, X, T, row0, h->stream);
    row0 += L.n[0] / 2 - 2 * RX_GUARD;
    e = hipGetLastError();
    if (e != hipSuccess) rc = fail_hip(e, "rx_train_mlp windows");
  }
  if (rc == RX_OK) e = hipStreamSynchronize(h->stream);
  h->hj.seed = seed0;
  h->hj.ref_ext = ext0;
  h->hj.mlp = mlp0;
  int rc2 = upload_job(h);
  if (rc == RX_OK) rc = rc2;
  if (rc == RX_OK) rc = rx_train_mlp_data(h, X, T, (size_t)rows, c, final_loss);
  hipFree(X);
  hipFree(T);
  h->stream_pos = 0;   // the training buffers replaced a stream's acquisition: it starts over
  h->acquired = false;
  return rc;
}

int rx_mlp_grad(rx_handle h, const float *dev_x, const float *dev_t, size_t n, float *dev_grad, double *loss_out) {
  if (!h || !dev_x || !dev_t || !dev_grad || n == 0 || n > 65536) return RX_E_INVALID;
  if (!h->mlp) return RX_E_UNSUPPORTED;
  if (!h->mlp_ready) return RX_E_STATE;
  const int np = rx_mlp_params();
  const int nwg = ((int)n + 63) / 64;
  float *part = nullptr;
  double *loss = nullptr;
  hipError_t e = hipMalloc(&part, (size_t)nwg * np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&loss, nwg * sizeof(double));
  if (e == hipSuccess) {
    rx_mlp_step(dev_x, dev_t, (int64_t)n, 0, (int)n, 0, h->mlp, nullptr, nullptr, part, loss, dev_grad, 0, 0.f, 0.f,
                0.f, 0.f, 1.f, 1.f, h->stream);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess && loss_out) {
    std::vector<double> lp(nwg);
    e = hipMemcpy(lp.data(), loss, nwg * sizeof(double), hipMemcpyDeviceToHost);
    double acc = 0.0;
    for (double x : lp) acc += x;
    *loss_out = acc / (double)n;
  }
  hipFree(part);
  hipFree(loss);
  return e == hipSuccess ? RX_OK : fail_hip(e, "rx_mlp_grad");
}

int rx_mlp_grad_static(rx_handle h, const float *dev_x, const float *dev_t, size_t n, float *dev_grad,
                       double *loss_out) {
  if (!h || !dev_x || !dev_t || !dev_grad || n == 0 || n > RX_MLP_STATIC_ROWS) return RX_E_INVALID;
  if (!h->mlp || !h->scratch) return RX_E_UNSUPPORTED;
  if (!h->mlp_ready) return RX_E_STATE;
  const int np = rx_mlp_params();
  const int nwg = ((int)n + 63) / 64;   // <= rx_mlp_scratch_parts()
  float *part = static_cast<float *>(h->scratch);
  double *loss = reinterpret_cast<double *>(part + (size_t)rx_mlp_scratch_parts() * np);
  rx_mlp_step(dev_x, dev_t, (int64_t)n, 0, (int)n, 0, h->mlp, nullptr, nullptr, part, loss, dev_grad, 0, 0.f, 0.f,
              0.f, 0.f, 1.f, 1.f, h->stream);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess && loss_out) {
    double lp[RX_MLP_STATIC_ROWS / 64];   // the partials, on the host stack
    e = hipMemcpy(lp, loss, nwg * sizeof(double), hipMemcpyDeviceToHost);
    double acc = 0.0;
    for (int i = 0; i < nwg; i++) acc += lp[i];
    *loss_out = acc / (double)n;
  }
  return e == hipSuccess ? RX_OK : fail_hip(e, "rx_mlp_grad_static");
}

int rx_mlp_infer(rx_handle h, const float *dev_x, size_t n, float *dev_y) {
  if (!h || !dev_x || !dev_y || n == 0) return RX_E_INVALID;
  if (!h->mlp) return RX_E_UNSUPPORTED;
  if (!h->mlp_ready) return RX_E_STATE;
  rx_mlp_infer_rows(h->mlp, dev_x, (int64_t)n, dev_y, h->stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? RX_OK : fail_hip(e, "rx_mlp_infer");
}

// Weights file: "RXMLP001", uint32 parameter count, float32 parameters (LE).
int rx_save_weights(rx_handle h, const char *path) {
  if (!h || !path) return RX_E_INVALID;
  const int np = rx_mlp_params();
  std::vector<float> w(np);
  int rc = rx_get_mlp(h, w.data());
  if (rc) return rc;
  FILE *f = std::fopen(path, "wb");
  if (!f) return RX_E_INVALID;
  const uint32_t cnt = (uint32_t)np;
  bool ok = std::fwrite("RXMLP001", 1, 8, f) == 8 && std::fwrite(&cnt, 4, 1, f) == 1 &&
            std::fwrite(w.data(), 4, np, f) == (size_t)np;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? RX_OK : RX_E_INVALID;
}

int rx_load_weights(rx_handle h, const char *path) {
  if (!h || !path) return RX_E_INVALID;
  const int np = rx_mlp_params();
  FILE *f = std::fopen(path, "rb");
  if (!f) return RX_E_INVALID;
  char magic[8];
  uint32_t cnt = 0;
  std::vector<float> w(np);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "RXMLP001", 8) == 0 &&
            std::fread(&cnt, 4, 1, f) == 1 && cnt == (uint32_t)np && std::fread(w.data(), 4, np, f) == (size_t)np;
  std::fclose(f);
  if (!ok) return RX_E_INVALID;
  return rx_set_mlp(h, w.data());
}

int rx_stage_times(rx_handle h, double *ms, uint64_t *launches, int max_stages) {
  if (!h || max_stages < 0) return RX_E_INVALID;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  for (auto &p : h->pending) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      h->stage_ms[p.stage] += t;
      h->stage_n[p.stage] += 1;
    }
    h->pool.push_back(p.a);
    h->pool.push_back(p.b);
  }
  h->pending.clear();
  if (!ms) {
    for (int i = 0; i < ST_COUNT; i++) { h->stage_ms[i] = 0.0; h->stage_n[i] = 0; }
    return ST_COUNT;
  }
  for (int i = 0; i < ST_COUNT && i < max_stages; i++) {
    ms[i] = h->stage_ms[i];
    if (launches) launches[i] = h->stage_n[i];
  }
  return ST_COUNT;
}

void rx_destroy(rx_handle h) {
  if (!h) return;
  hipStreamSynchronize(h->stream);
  if (h->graph.exec) hipGraphExecDestroy(h->graph.exec);
  if (h->graph.capture) hipStreamDestroy(h->graph.capture);
  delete h;
}

}  // extern "C"

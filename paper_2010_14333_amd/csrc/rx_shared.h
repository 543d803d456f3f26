// Declarations shared by the host library and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RX_MAXB 64          // buffers per batched launch
#define RX_PREFIX_MAX 4096  // longest known prefix the prefix kernel holds in LDS
#define RX_GUARD 64         // symbols excluded at each end of the error-count window
#define RX_LAG 64           // delay search range [-RX_LAG, RX_LAG] symbols
#define RX_KMAX 32          // tap storage per handle
#define RX_LAT_RING 1024    // per-buffer latencies a handle keeps (the most recent)

// Per-buffer scalars written by the kernels (device memory, one per handle).
struct RxScalars {
  double mean_re, mean_im;  // KK carrier mean / PAM mean of v
  double agc;               // unit-power gain
  double theta0;            // static carrier phase of the CMA taps (KK)
  int32_t lag, rot, fallback, pad;
  float2 w0[RX_KMAX];       // prefix FFE taps
  unsigned long long stats[7];  // buffers, symbols, bits, bit errors, symbol errors, fallbacks,
                                // buffers later than their deadline
  unsigned long long t_start;   // wall-clock ticks when the buffer's first workgroup started
  unsigned int done_wg;         // decision workgroups of the current buffer that have finished
  unsigned int kk_next;         // KK front end: work items handed out beyond the first grid (launch job 0)
  unsigned int kk_done, pad2;   // KK front end: workgroups that found the queue empty (launch job 0)
  unsigned long long lat_count; // buffers whose latency has been recorded
  unsigned int lat[RX_LAT_RING];   // latency (ticks) of recorded buffer i at index i % RX_LAT_RING
  double theta_carry;           // stream: KK carrier phase of the last emitted DD-LMS block
  double acc_carry;             // stream: PAM unwrapped timing angle of the last emitted timing block
};

// Everything a kernel needs about one handle (device memory, written once).
struct RxJob {
  int32_t fmt, kk, bps, m_axis;     // format, KK flag, bits/symbol, levels per real axis
  int32_t mf_taps, ffe_taps, prefix, precision;
  int32_t fft_log2, hop, blk, equalizer;  // KK OS geometry, DD-LMS block length
  float mu, mu_cma, r2, ea2_sqrt;   // steps, CMA radius, sqrt(E|a|^2)
  double r;                         // carrier offset / fs (signed)
  float sgn;                        // Hilbert sign (+1: signal above the carrier)
  int32_t debug;                    // keep derotated soft symbols
  int32_t ref_ext;                  // known symbols from the caller's reference stream (refw), not the seed
  int32_t stream;                   // contiguous stream: decisions held back by `hold` samples
  int32_t hold, look;               // stream: hold-back and look-back (samples) of the prepended tail
  uint64_t ref_period;              // the reference sequence repeats every ref_period symbols (0: never)
  uint64_t seed;
  float2 c0;                        // interior value of MF(exp(-j 2 pi r n)) / exp(-j 2 pi r 2m)
  const float *mf;                  // matched filter taps (65 centred for KK, 33 for PAM)
  const float *hspec;               // KK: Hilbert spectrum sgn S[k] c / N (H = -j S; c = (ln 2 / 2) / (2 pi):
                                    //   the transforms take log2 v and give the phase in revolutions), N
                                    //   entries, then (N = 2^14) the same in the 16 x 1024 transform's order
  const float2 *twid;               // KK: exp(-j 2 pi k / N), N entries, then exp(-j 2 pi k / 1024), 1024
  float2 *z;                        // KK: MF output / carrier-free field at 2 sps [n/2]
  float *y;                         // PAM: MF output [n]
  float *xr;                        // PAM: timing-corrected samples [n]
  double2 *part;                    // per-workgroup partial sums (KK: 3 per workgroup, see kk_front)
  double *part2;                    // per-workgroup partial sums (stage 2)
  uint32_t *upart;                  // PAM code-sum partials
  float2 *gard;                     // PAM: Gardner sums per 512-sample block
  float *delta;                     // PAM: timing shift per block (samples)
  float2 *soft;                     // soft symbols: KK float2, PAM packed floats (read as float[])
  float2 *s4;                       // KK: sum z^4 per DD-LMS block
  float *theta;                     // KK: carrier phase per block
  float2 *field;                    // KK debug: reconstructed field [n] or null
  float2 *udbg;                     // KK debug: AGC'd carrier-free MF output [n/2] or null
  float *phi;                       // KK frequency-domain front end: phase (revolutions) [n]
  double2 *fdpart;                  // KK frequency-domain front end: field sums per block pair
  int32_t dd_phase;                 // KK: the DD-LMS taps carry the carrier phase (no VV stage)
  int32_t pad_dd;
  const float *mlp;                 // PAM learned equaliser parameters (FP32) or null
  const uint32_t *refw;             // reference bits of symbols 0 .. max_samples / sps - 1, packed as the output
  RxScalars *sc;
  double deadline_ticks;            // > 0: latency budget of every buffer in wall-clock ticks
  double ticks_per_sample;          // otherwise the budget is n / fs: wall-clock ticks per input sample
};

// By-value launch description of one batch (kernel argument, < 4 KiB).
// s0[i] >= 0 marks a stream buffer after the first: its input is the stream's
// previous `hold + look` samples followed by the new buffer, and s0 is the
// stream index of its first sample; -1 for an independent buffer or the
// first buffer of a stream.
struct RxLaunch {
  const RxJob *job[RX_MAXB];
  const uint8_t *in[RX_MAXB];
  uint8_t *bits[RX_MAXB];
  int64_t n[RX_MAXB];
  int64_t s0[RX_MAXB];
  int32_t count;
  int32_t pad;
};

// Hold-back (decisions of the last `hold` samples of a stream buffer wait for
// the next buffer) and look-back (samples before the first emitted one that
// the chain needs) of the contiguous-stream mode, per chain: the KK chain's
// Hilbert and matched-filter reach, FFE span and delay, DD-LMS block and
// carrier-phase window fit in 4096 samples either way; the PAM chain's
// timing-detector averaging window (16 blocks of 512) sets 12288.
#define RX_KK_HOLD 4096
#define RX_PAM_HOLD 12288
// Symbol ranges of a launch entry, in symbols of its processed input.
struct RxSpan {
  int64_t k_lo, k_hi;   // emitted symbols [k_lo, k_hi) (output bit 0 = symbol k_lo)
  int64_t g0;           // stream index of the input's first sample (0 unless continuing a stream)
  int64_t kg0;          // stream symbol index of the input's first symbol
};
__host__ __device__ inline RxSpan rx_span(const RxJob &J, int64_t n, int64_t s0) {
  const int sps = J.kk ? 4 : 2;
  RxSpan sp;
  sp.g0 = s0 > 0 ? s0 : 0;
  sp.kg0 = sp.g0 / sps;
  sp.k_lo = (J.stream && s0 >= 0) ? J.look / sps : 0;
  sp.k_hi = J.stream ? (n - J.hold) / sps : n / sps;
  return sp;
}

// KK overlap-save geometry: a frame of N samples starts RX_KK_EDGE samples
// before its hop, the Hilbert FIR reaches 2048 samples either side and the
// matched filter 32 more; hop is what remains, rounded down to 16 samples.
#define RX_KK_HALFV 2048
#define RX_KK_CMF 32
#define RX_KK_EDGE 2080
static inline int rx_kk_hop(int log2n) {
  int h = (1 << log2n) - RX_KK_HALFV - RX_KK_EDGE - RX_KK_CMF;
  return h & ~15;
}

// Launch shapes picked per (GPU, chain, precision, FFE length) by the
// library's tuner: overlap-save FFT size, DD-LMS chunk steps, precision-form
// FFE groups per wavefront, decision symbols per workgroup.  Every choice
// computes the same result (the FFT size up to rounding).
struct RxTune {
  int32_t fft_log2, blocks_bc, ffe_gpw, dec_syms;
};

// Kernel stages (host-side launchers are defined with their kernels).
enum RxStage {
  ST_KK_FRONT = 0, ST_KK_DEBUG, ST_PAM_SUM, ST_PAM_MF, ST_PAM_GAVG, ST_PAM_UNWRAP, ST_PAM_FARROW,
  ST_PREFIX, ST_BLOCKS, ST_KK_VV, ST_DECIDE, ST_MLP_INFER, ST_MLP_JUDGE, ST_COUNT
};
void rx_launch_kk_stage(int stage, const RxLaunch &L, int64_t maxn, int log2n, int prec, hipStream_t s);
// the paper's frequency-domain KK front end (jobs with fft_log2 == RX_KK_FD_LOG2)
#define RX_KK_FD_LOG2 10
void rx_launch_kkfd(const RxLaunch &L, int64_t maxn, hipStream_t s);
// the paper's frequency-domain PAM static equaliser (stage ST_PAM_MF) and
// clock recovery (ST_PAM_FARROW), for jobs with fft_log2 == RX_KK_FD_LOG2
void rx_launch_pamfd(int stage, const RxLaunch &L, int64_t maxn, hipStream_t s);
void rx_launch_pam_stage(int stage, const RxLaunch &L, int64_t maxn, int log2n, hipStream_t s);
void rx_launch_eq_stage(int stage, const RxLaunch &L, int64_t maxn, int kk, int ffe_taps, int prec, const RxTune &t,
                        hipStream_t s);
void rx_launch_mlp_stage(int stage, const RxLaunch &L, int64_t maxn, hipStream_t s);
void rx_launch_ref_fill(uint32_t *w, int64_t words, uint64_t seed, int bps, int64_t nsym, uint64_t period,
                        hipStream_t s);
void rx_mlp_windows(const RxLaunch &L, float *X, float *T, int64_t row0, hipStream_t s);
int rx_mlp_params(void);
void rx_mlp_step(const float *X, const float *T, int64_t ntrain, int64_t i0, int batch, int64_t mult, float *p,
                 float *m, float *v, float *part, double *loss_part, float *grad, int adam, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t s);
void rx_mlp_infer_rows(const float *P, const float *X, int64_t n, float *Y, hipStream_t s);
#define RX_MLP_STATIC_ROWS 8192   // rows rx_mlp_grad_static takes (its partials live in a static array)
int rx_mlp_scratch_resolve(void **out);   // 0 or a hipError_t
int rx_mlp_scratch_parts(void);

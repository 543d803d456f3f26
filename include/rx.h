/*
 * rx.h -- C ABI of the MI355X receiver library (librx.so).
 *
 * The library implements the per-buffer DSP hot path of a software-defined,
 * GPU-based optical receiver (van der Heide et al., ECOC 2020): a buffer of
 * 12-bit ADC samples in device memory goes in, hard-decision bits and error
 * counts come out.  Two chains, selected at create time (the paper switches
 * formats by changing only the GPU software, Sec. 1, second paragraph):
 *
 *   - PAM-2/4/8 at 2 samples/symbol: DC removal, matched filter, blockwise
 *     clock-phase estimation + unwrapping + clock recovery, FFE, decision,
 *     demapping (Sec. 2, first paragraph);
 *   - Kramers-Kronig QPSK/16QAM at 4 samples/symbol: sqrt/log, FFT
 *     Hilbert transform, field recovery and frequency downshift (Fig. 1d),
 *     filtering and decimation to 2 samples/symbol, adaptive FFE with clock-
 *     and symbol-phase recovery, decision, demapping (Sec. 2, second
 *     paragraph).
 *
 * Conventions shared by every entry point
 *   - Return value: 0 on success, a negative RX_E_* code on error, or the
 *     positive warning RX_W_FALLBACK.  No C++ exception crosses the ABI.
 *   - Pointers named dev_* are device (HBM) pointers owned by the caller; they
 *     must stay valid until the handle's stream has passed the enqueued work
 *     (rx_errors() or a stream synchronisation).  The library owns every
 *     workspace it allocates and frees it in rx_destroy().
 *   - Work is enqueued asynchronously on the handle's stream.  Handles are not
 *     thread-safe: use one handle per host thread.
 *   - Input layout: n_samples unsigned 12-bit codes, two per three bytes,
 *     little-endian (byte0 = s0 & 0xFF, byte1 = (s0 >> 8) | ((s1 & 0xF) << 4),
 *     byte2 = s1 >> 4); n_samples is a multiple of 1024.  Code c is read as
 *     the photocurrent c + 0.5 (Sec. 2, first paragraph: 2^22 12-bit samples
 *     per buffer at 4 Gs/s).
 *   - Output bits: symbol-major, Gray bits MSB-first within a symbol; stream
 *     bit t lives in byte t >> 3 at bit position t & 7 (LSB first).  The
 *     kernels write whole 32-bit words of it.
 *   - Alignment: dev_buffer and dev_bits (and ref_bits) must be 4-byte
 *     aligned (the kernels read and write 32-bit words); a misaligned
 *     pointer is rejected with RX_E_INVALID before anything is enqueued.
 *     Host pointers of rx_process_batch_host need no alignment.
 */
#ifndef RX_H
#define RX_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rx_ctx *rx_handle;

typedef enum { RX_PAM2 = 1, RX_PAM4 = 2, RX_PAM8 = 3, RX_KK_QPSK = 4, RX_KK_16QAM = 5 } rx_format;
typedef enum { RX_FP32 = 0, RX_BF16 = 1, RX_FP16 = 2 } rx_precision;
typedef enum { RX_EQ_LMS = 0, RX_EQ_MLP = 1 } rx_equalizer;
/* KK front end.  RX_FRONT_OS: a finite 4097-tap Hilbert FIR applied by
 * overlap-save FFTs and the 65-tap matched filter on MFMA.  RX_FRONT_FD: the
 * paper's own frequency-domain form (Sec. 2, second paragraph, with the first
 * paragraph's 1024-point "100 % overlap" blocks): 1024-point blocks advancing
 * by 512 samples, the Hilbert transform as -j sgn(k) on each block's
 * spectrum, field and FP64-phase downshift with the carrier mean removed,
 * the 203-tap static equaliser on the 1024-point spectrum (the matched RRC:
 * the paper's taps are unpublished and their link-specific part is the
 * identity back to back), the 512 bins of |f| < fs/4 through a 512-point
 * inverse transform to 2 samples per symbol.  FP32, independent buffers
 * only; mf_taps, hilbert_taps and fft_log2 do not apply to it. */
typedef enum { RX_FRONT_OS = 0, RX_FRONT_FD = 1 } rx_front;

enum {
  RX_OK = 0,
  RX_E_INVALID = -1,      /* bad argument or unsupported size / rate */
  RX_E_UNSUPPORTED = -2,  /* combination not provided (e.g. MLP on a KK format) */
  RX_E_NOMEM = -3,        /* device allocation failed */
  RX_E_HIP = -4,          /* a HIP call failed; rx_strerror() gives the HIP text */
  RX_E_STATE = -5,        /* call-order violation (e.g. MLP inference before weights) */
  RX_W_FALLBACK = 1       /* warning: the MLP lost to LMS on the known prefix; LMS ran */
};

/* Flags */
#define RX_DEBUG_KEEP 0x1u   /* keep intermediate arrays for rx_debug_fetch() */
#define RX_PROFILE 0x2u      /* time every kernel stage with HIP events (see rx_stage_times) */
#define RX_STREAM 0x4u       /* the handle's buffers are consecutive pieces of one continuous stream
                                (see "Contiguous streams" below) */
#define RX_DD_PHASE 0x8u     /* KK: no Viterbi-Viterbi carrier-phase stage; the block DD-LMS taps,
                                started from the prefix acquisition, carry the carrier phase (the
                                paper's short DD-LMS doing clock- and symbol-phase recovery, Sec. 2,
                                second paragraph; with ffe_taps = 4 its 4-tap form).  PAM:
                                RX_E_UNSUPPORTED */

/* Kernel stages reported by rx_stage_times (index into its arrays). */
enum {
  RX_ST_KK_FRONT = 0,   /* unpack, ln, FFT Hilbert, field, FP64 downshift, decimating MF */
  RX_ST_KK_DEBUG,       /* (RX_DEBUG_KEEP only) materialises the AGC'd carrier-free MF output */
  RX_ST_PAM_SUM,        /* exact code sum (DC) */
  RX_ST_PAM_MF,         /* DC removal, matched filter, timing-detector sums */
  RX_ST_PAM_GAVG,       /* timing-detector averaging and angle */
  RX_ST_PAM_UNWRAP,     /* timing unwrap, AGC gain */
  RX_ST_PAM_FARROW,     /* cubic interpolation onto the recovered clock */
  RX_ST_PREFIX,         /* (CMA,) delay search, LMS training on the known prefix */
  RX_ST_BLOCKS,         /* block-parallel DD-LMS FFE */
  RX_ST_KK_VV,          /* Viterbi-Viterbi block phase, unwrap */
  RX_ST_DECIDE,         /* decisions, demapping, packing, error counting */
  RX_ST_MLP_INFER,      /* learned equaliser, BF16 MFMA inference */
  RX_ST_MLP_JUDGE,      /* MLP vs LMS errors on the known prefix (sets the fallback) */
  RX_NSTAGES
};

typedef struct {
  uint32_t struct_size;     /* sizeof(rx_params), for ABI evolution */
  int32_t mf_taps;          /* matched RRC length: 33 (PAM, 2 sps), 65 (KK, 4 sps); odd, at most
                               33 (PAM) / 65 (KK); shorter filters are centred in those slots */
  int32_t ffe_taps;         /* T/2-spaced FFE length: 15 (PAM), 21 (KK); 15 or 21 for either chain,
                               or 4 for KK (the paper's 4-tap DD-LMS; tap i multiplies sample
                               2k + (K - 1) / 2 - i of symbol k, integer division); the precision
                               form: 21 */
  int32_t prefix_symbols;   /* known training/sync symbols at each buffer start: 4096 */
  int32_t hilbert_taps;     /* KK Hilbert FIR length V+1: 4097 */
  int32_t fft_log2;         /* KK overlap-save FFT size: 0 = tuned, else 13 or 14 */
  int32_t precision;        /* rx_precision: RX_FP32 plain chain; BF16/FP16 precision form (KK) */
  int32_t equalizer;        /* rx_equalizer (MLP: PAM only) */
  double rolloff;           /* RRC roll-off: 0.1 */
  double mu;                /* LMS / DD-LMS step: 1e-3 */
  double mu_cma;            /* CMA step (KK): 1e-3 */
  double carrier_hz;        /* KK tone offset, signed: +0.55e9 = signal above the carrier */
  uint64_t seed;            /* reference sequence: bits of symbol k are the top log2(M) bits
                               of the k-th SplitMix64 output seeded with `seed` */
  uint64_t max_samples;     /* largest n_samples a call may pass (sizes the workspace) */
  void *stream;             /* hipStream_t for all work of this handle; NULL = null stream */
  uint32_t flags;           /* RX_DEBUG_KEEP, RX_PROFILE */
  uint32_t reserved;
  double deadline_s;        /* latency budget of every buffer, seconds; 0 = the buffer's own
                               real-time span n_samples / fs (Sec. 2, first paragraph: each
                               buffer processed before the next ones arrive); see rx_latencies */
  const void *ref_bits;     /* NULL: the reference stream comes from `seed`.  Else a device
                               pointer, owned by the caller, to the reference bits of symbols
                               0 .. max_samples / sps - 1 packed like the output bits (4-byte
                               aligned, at least 4 * ceil(max_samples / sps * log2(M) / 32)
                               bytes, valid while the handle processes buffers).  Both the
                               known prefix (training, delay search) and the error count read
                               it, while the buffer's kernels run, so a caller processing
                               buffers of different sequences on one handle rewrites it on
                               the handle's stream between them.  rx_train_mlp still takes
                               its training buffers' sequences from its seeds.  Not with
                               RX_STREAM (RX_E_UNSUPPORTED). */
  uint64_t ref_period;      /* 0, or the seeded reference sequence repeats every ref_period
                               symbols (symbol k is that of k mod ref_period), as the pattern
                               of a transmitter that repeats a finite memory */
  int32_t blocks_bc;        /* DD-LMS symbol steps per staged chunk: 4, 8 or 16; 0 = tuned */
  int32_t ffe_gpw;          /* precision-form FFE: 256-symbol groups per wavefront: 4, 8 or 16;
                               0 = tuned */
  int32_t dec_syms;         /* decision stage: symbols per workgroup: 1024, 2048 or 4096; 0 = tuned */
  int32_t front;            /* rx_front (KK): RX_FRONT_OS (default) or RX_FRONT_FD; RX_FRONT_FD
                               with a PAM format, a precision form or RX_STREAM:
                               RX_E_UNSUPPORTED */
} rx_params;

/* Cumulative counters since create / rx_errors_reset.  Symbols counted are
 * those in [prefix + 64, n_symbols - 64) of each buffer (Sec. 3, second
 * paragraph: Q-factor estimated from the error rate).  late_buffers counts
 * buffers whose latency (rx_latencies) exceeded the handle's deadline. */
typedef struct {
  uint64_t buffers, symbols, bits, bit_errors, symbol_errors, fallbacks, late_buffers;
} rx_stats;

/* Debug stages for rx_debug_fetch (the handle needs RX_DEBUG_KEEP for FIELD). */
enum {
  RX_STAGE_FIELD = 1,   /* KK: reconstructed field E, float2[n] (needs RX_DEBUG_KEEP) */
  RX_STAGE_MF = 2,      /* KK: AGC'd carrier-free decimated MF output float2[n/2] (needs RX_DEBUG_KEEP);
                           PAM: MF output before the AGC gain, float[n] */
  RX_STAGE_XR = 3,      /* PAM: timing-corrected samples float[n] */
  RX_STAGE_TIMING = 4,  /* PAM: timing shift (samples) per 512-sample block, float[n/512] */
  RX_STAGE_SOFT = 5,    /* soft symbols after carrier phase (KK float2, PAM float) [n_sym] */
  RX_STAGE_TAPS = 6,    /* prefix FFE taps w0, float2[ffe_taps] */
  RX_STAGE_PHASE = 7,   /* KK: unwrapped carrier phase per 128-symbol block, float[n_sym/128] */
  RX_STAGE_SCALARS = 8  /* double[8]: mean re, mean im, agc, theta0, lag, rot, fallback, 0 */
};

/* Launch shapes.  fft_log2, blocks_bc, ffe_gpw and dec_syms change how the
 * work is laid out on the GPU, never the result (the FFT size changes it by
 * rounding only: the Hilbert transform is a fixed finite kernel).  Left at
 * 0 they are tuned on the device: the first rx_create of a (GPU
 * architecture, chain, precision, FFE length) times each stage with each
 * candidate on a 16-buffer batch (about a second) and keeps the fastest;
 * the choices are cached for the process and in a JSON file
 * ($RX_TUNE_CACHE, else $HOME/.cache/paper_2010_14333_amd/autotune.json;
 * RX_TUNE_CACHE="" keeps them in memory only).  rx_tuning reports a
 * handle's shapes: shapes[0..3] = fft_log2, blocks_bc, ffe_gpw, dec_syms. */
int rx_tuning(rx_handle h, int32_t *shapes);

/* Fill *p with the defaults of `fmt` (values in the comments above).
 * Returns RX_E_INVALID for an unknown format or NULL p. */
int rx_params_default(rx_format fmt, rx_params *p);

/* Create a receiver for one format (Sec. 1, second paragraph: the format is
 * selected in software).  baud/fs must be 2e9/4e9 (PAM) or 1e9/4e9 (KK),
 * i.e. 2 and 4 samples per symbol.  Designs the filters in FP64 on the host,
 * rounds them once, allocates the workspace for p->max_samples, and writes
 * the reference bits of every symbol a buffer can hold (max_samples / sps
 * symbols of log2(M) bits, from the seed) once, on the null stream, before
 * returning: every buffer of the handle is counted against them.
 * p may be NULL (defaults).  On success *out owns device memory. */
int rx_create(rx_format fmt, double baud, double fs, const rx_params *p, rx_handle *out);

/* Process one buffer (Fig. 1a: buffer in, bits out).  dev_buffer holds
 * n_samples packed 12-bit codes (1.5 * n_samples bytes); dev_bits receives
 * ceil(n_sym * log2(M) / 8) bytes, n_sym = n_samples / sps.  *n_bits_out (may
 * be NULL) is set on the host without synchronising.  Asynchronous on the
 * handle's stream.  Errors: RX_E_INVALID if a pointer is NULL or not 4-byte
 * aligned, if n_samples is not a positive multiple of 1024, exceeds
 * max_samples, or leaves fewer than prefix + 128 symbols; RX_E_HIP on a
 * launch failure. */
int rx_process(rx_handle h, const void *dev_buffer, size_t n_samples, void *dev_bits,
               size_t *n_bits_out);

/* Contiguous streams (RX_STREAM).  The ADC delivers one continuous stream
 * of buffers and the receiver keeps the signal continuous across them (Sec.
 * 2, first paragraph: each overlap-and-save kernel prepends part of the
 * previous buffer, and the blockwise clock-phase unwrap continues from the
 * previous buffer).  On a stream handle:
 *   - the first buffer (after create or rx_stream_reset) is processed as an
 *     independent buffer and acquires the stream: carrier (KK) or DC (PAM)
 *     mean, AGC gain, static phase, symbol delay, rotation, prefix taps and
 *     the network's judgement are those of this buffer for the whole stream;
 *     the known prefix is only at the stream's start;
 *   - every later buffer is processed after the stream's preceding
 *     hold + look samples (hold = look = 4096 samples KK, 12288 PAM), with the
 *     downshift phase taken at the stream's sample index, the DD-LMS blocks
 *     on the stream's grid, and the KK carrier-phase and PAM clock-phase
 *     unwraps continued from the previous buffer's last emitted block;
 *   - decisions are emitted `hold` samples late: the first buffer emits the
 *     symbols of its first n - hold samples, each later one exactly n / sps
 *     symbols (the previous buffer's held-back samples first), so the output
 *     bits of consecutive calls concatenate into the stream's bits and no
 *     emitted decision depends on samples not yet received;
 *   - errors count the stream's symbols from prefix + 64 on (reference
 *     symbol = the stream's symbol index, mod ref_period when set).
 * The call's dev_buffer must hold n packed samples as usual (any multiple of
 * 1024 after the first; the first must hold the prefix plus hold + look
 * samples); it is copied into the handle's staging area (the library keeps
 * the tail), so it may be reused once the handle's stream has passed the
 * call.  *n_bits_out reports the emitted bits.  Graph replay is not offered
 * for stream handles (their launch arguments change every call:
 * RX_E_UNSUPPORTED).  rx_train_mlp on a stream handle restarts its stream. */
int rx_stream_reset(rx_handle h);   /* the next buffer starts (and acquires) a new stream; RX_E_STATE
                                       on a handle without RX_STREAM */

/* Process `count` buffers (1..64) with distinct handles, mixed formats
 * allowed, as one batched launch sequence on the FIRST handle's stream (the
 * paper overlaps 5 buffers on 5 streams, Sec. 2, first paragraph; here all
 * buffers share every kernel launch).  With graph != 0 the launch sequence
 * is captured once (on a library-owned stream) into a hipGraph per (handles,
 * buffers, sizes) and replayed on the first handle's stream.
 * A cached graph is replayed only for the same handles (by a process-unique
 * id, not their addresses) in the same state: setting or training a
 * handle's network, or destroying and re-creating handles, leads to a new
 * capture.  Arguments as for rx_process, one entry per buffer.  Errors:
 * RX_E_INVALID for count outside 1..64, a repeated handle, handles on
 * different streams, or a pointer that rx_process rejects. */
int rx_process_batch(const rx_handle *hs, const void *const *dev_buffers, const size_t *n_samples,
                     void *const *dev_bits, int count, int graph);

/* Host-resident buffers, as the paper's receiver takes them: the ADC board
 * writes each buffer into host memory and the host moves it to the GPU
 * (Fig. 1a; Sec. 2, first paragraph).  Copies host_buffers[i] (n_samples[i]
 * packed codes, 1.5 * n_samples[i] bytes) into a device staging area of
 * handle i, runs the batch as rx_process_batch does, and copies the bits
 * back into host_bits[i] (size as for rx_process); everything is enqueued
 * on the FIRST handle's stream and the call returns without waiting.  The
 * host buffers must stay valid, and host_bits must not be read, until that
 * stream is synchronised (rx_sync or rx_errors).  Pinned host memory
 * (hipHostMalloc) lets the copies run asynchronously and overlap work on
 * other streams; pageable memory is accepted but its copies block the
 * caller.  Each handle's staging area (1.5 * max_samples bytes in, the bits
 * of max_samples out) is allocated by the library on the handle's first
 * such call and freed by rx_destroy.  Errors: as rx_process_batch;
 * RX_E_NOMEM if a staging area cannot be allocated; RX_E_HIP if a copy
 * cannot be enqueued. */
int rx_process_batch_host(const rx_handle *hs, const void *const *host_buffers, const size_t *n_samples,
                          void *const *host_bits, int count, int graph);

/* Wait for all work enqueued on the handle's stream. */
int rx_sync(rx_handle h);

/* Synchronise the handle's stream and copy the cumulative counters. */
int rx_errors(rx_handle h, rx_stats *out);
/* Zero the counters and the latency record. */
int rx_errors_reset(rx_handle h);

/* Per-buffer latency, measured on the device (the paper's real-time
 * criterion, Sec. 2, first paragraph: every buffer processed within its
 * budget): the wall clock when the buffer's first kernel starts its first
 * workgroup, to when its last decision workgroup finishes; compared with the
 * deadline (rx_params.deadline_s, else n_samples / fs) into
 * rx_stats.late_buffers.  Copies the latencies, in microseconds, of the
 * most recent min(recorded, 1024, max) buffers of this handle, oldest first,
 * into us[] and their number into *count (may be NULL); synchronises the
 * handle's stream.  In a batch, a buffer's latency includes the other
 * buffers it shares each launch with. */
int rx_latencies(rx_handle h, double *us, size_t max, size_t *count);

/* Copy an intermediate array of the most recent buffer to host memory
 * (synchronises).  bytes must equal the stage's size for that buffer.
 * RX_E_STATE if nothing was processed or the stage needs RX_DEBUG_KEEP. */
int rx_debug_fetch(rx_handle h, int stage, void *host_dst, size_t bytes);

/* ---- Learned equaliser (PAM formats, equalizer = RX_EQ_MLP) ------------
 * A 31 -> 64 ReLU -> 64 ReLU -> 1 network over the 31 timing-corrected
 * samples centred on each symbol replaces the block DD-LMS FFE (the paper's
 * PAM chain equalises with an LMS FFE, Sec. 2, first paragraph).  It is
 * trained in FP32 by the library's own forward/backward/Adam kernels and
 * runs as BF16 MFMA inference.  LMS stays the fallback and the judge: per
 * buffer, if the network makes more decision errors than the LMS taps on
 * the known prefix, the block DD-LMS runs instead (counted in
 * rx_stats.fallbacks).  rx_process on an MLP handle without weights runs
 * LMS and returns RX_W_FALLBACK.
 * Parameters: RX_MLP_PARAMS floats packed W1[64][31], b1[64], W2[64][64],
 * b2[64], W3[64], b3. */
#define RX_MLP_PARAMS 6273

typedef struct {
  uint32_t struct_size;   /* sizeof(rx_train_cfg) */
  int32_t epochs;         /* 2 */
  int32_t batch;          /* minibatch: 1024 */
  int32_t max_steps;      /* 0 = epochs * floor(n / batch) steps, else at most this many */
  double lr, beta1, beta2, eps;   /* Adam: 1e-3, 0.9, 0.999, 1e-8 */
  uint64_t init_seed;     /* Kaiming-uniform start drawn from SplitMix64(init_seed) if init is NULL */
  const float *init;      /* host pointer to RX_MLP_PARAMS start values, or NULL */
} rx_train_cfg;

int rx_train_cfg_default(rx_train_cfg *c);
int rx_mlp_param_count(void);
/* Row order of training: step t uses rows (mult * (t * batch + e)) mod n,
 * e < batch, mult = this value (the first odd number >= 1000003 coprime to n). */
int rx_mlp_order_multiplier(int64_t n);

/* Train on training buffers whose reference sequences have seeds[i]: each
 * buffer runs the PAM front end and prefix stage, every symbol in
 * [64, n_sym - 64) becomes one (window, level) row, then Adam on all rows.
 * Synchronous.  *final_loss (may be NULL) = last minibatch MSE.
 * RX_E_UNSUPPORTED on KK handles. */
int rx_train_mlp(rx_handle h, const void *const *dev_buffers, const size_t *n_samples, const uint64_t *seeds,
                 int count, const rx_train_cfg *c, double *final_loss);
/* Train on a given set: dev_x = n rows of 32 floats (31 samples + 0),
 * dev_t = n target levels (device memory).  Synchronous. */
int rx_train_mlp_data(rx_handle h, const float *dev_x, const float *dev_t, size_t n, const rx_train_cfg *c,
                      double *final_loss);
/* Gradient of (1/n) sum (y - t)^2 at the handle's weights over n <= 65536
 * rows (device x, t as above) into dev_grad[RX_MLP_PARAMS].  Synchronous. */
int rx_mlp_grad(rx_handle h, const float *dev_x, const float *dev_t, size_t n, float *dev_grad, double *loss);
/* rx_mlp_grad for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result, but the per-workgroup gradient partials live
 * in a static device array of the library (3.1 MiB per GPU, held until the
 * process ends) instead of memory allocated per call, so the call allocates
 * nothing.  n <= 8192 rows (RX_E_INVALID beyond that limit); the caller
 * passes x, t and dev_grad as for rx_mlp_grad; *loss (may be NULL) as
 * there.  Synchronous.  Every call on one GPU shares that GPU's array, which
 * keeps the last call's partials (each call overwrites all it reads):
 * calls that overlap on one GPU, from several threads or on several
 * streams, race.  RX_E_UNSUPPORTED on KK handles, RX_E_STATE before the
 * handle has weights. */
int rx_mlp_grad_static(rx_handle h, const float *dev_x, const float *dev_t, size_t n, float *dev_grad,
                       double *loss);
/* BF16 MFMA inference (the kernel of the chain's MLP stage) on given rows:
 * dev_x = n rows of 32 floats (column 31 ignored), dev_y = n outputs.  All
 * three layers' operands (inputs, weights, ReLU'd hidden activations) are
 * rounded to BF16 and their products summed in FP32; biases are added in
 * FP32.  Asynchronous. */
int rx_mlp_infer(rx_handle h, const float *dev_x, size_t n, float *dev_y);
/* Copy weights in/out (host memory), or to/from a file ("RXMLP001", uint32
 * count, float32 little-endian). */
int rx_set_mlp(rx_handle h, const float *host_params);
int rx_get_mlp(rx_handle h, float *host_params);
int rx_save_weights(rx_handle h, const char *path);
int rx_load_weights(rx_handle h, const char *path);

/* Stage timing of handles created with RX_PROFILE: synchronises the stream
 * and returns, per stage, the accumulated milliseconds and launch count of
 * every launch this handle led (it was the first handle of its batch) since
 * the last reset.  ms == NULL resets.  Returns RX_NSTAGES.  Graph replays are
 * not timed. */
int rx_stage_times(rx_handle h, double *ms, uint64_t *launches, int max_stages);

void rx_destroy(rx_handle h);
const char *rx_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif

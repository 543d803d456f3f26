/*
 * rxo.h -- FP64 CPU oracle of the software-defined receiver's two DSP chains.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; the two meet only
 * at the seeded synthetic inputs.
 *
 * Everything is computed in double precision, single-threaded, in the order
 * the chain is defined (no blocking or fusion beyond what a definition states).
 */
#ifndef RXO_H
#define RXO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { RXO_PAM2 = 1, RXO_PAM4, RXO_PAM8, RXO_KK_QPSK, RXO_KK_16QAM };

typedef struct {
  int32_t fmt;           /* RXO_* */
  int32_t mf_taps;       /* matched RRC length: 33 (PAM, 2 sps) / 65 (KK, 4 sps) */
  int32_t ffe_taps;      /* T/2-spaced FFE length: 15 (PAM) / 21 (KK), or 4 (the paper's KK
                            DD-LMS); tap i multiplies x[2k + (K - 1) / 2 - i] (integer division) */
  int32_t prefix;        /* known training/sync symbols at the buffer start */
  int32_t hilbert_taps;  /* odd: V+1 */
  int32_t os_log2;       /* FFT size of the oracle's own overlap-save (any >= log2(2V)) */
  int32_t form;          /* 0: block-parallel DD-LMS FFE; 1: FFE frozen at the prefix taps */
  int32_t rounding;      /* 0: none; 1: BF16; 2: FP16 operands (MF + FFE, or the MLP) */
  int32_t equalizer;     /* 0: LMS FFE; 1: MLP (PAM only) */
  int32_t front;         /* 0: the time-domain front end (KK: a finite Hilbert FIR by
                            overlap-save and the matched FIR; PAM: the matched FIR and cubic
                            Farrow timing correction).  1: the paper's frequency-domain form
                            on 1024-point blocks at hop 512 (KK: rxo_hilbert_fd, block-circular
                            Hilbert, and rxo_fd_eq_dec2, 203-tap static equaliser and
                            512-point IFFT to 2 sps; PAM: rxo_fd_fir, 503-tap static
                            equaliser, and rxo_fd_delay, timing correction in the frequency
                            domain).  FP64 arithmetic, one buffer, no learned equaliser */
  double rolloff, mu, mu_cma, fc_over_fs;
  uint64_t seed;         /* reference sequence: bits of symbol k = top bits of SplitMix64(seed, k) */
  const double *mlp;     /* RXO_MLP_PARAMS packed parameters when equalizer == 1 */
  const int32_t *force;  /* optional, nsym entries: decision index the block DD-LMS takes at that
                            symbol instead of its own (-1: its own); test instrumentation */
  const struct rxo_out_s *frozen;   /* optional: the acquisition of a stream (the result of its
                            first buffer): its means, AGC gain, static phase, delay, rotation,
                            prefix taps and MLP fallback are used instead of being computed */
  int64_t count_end;     /* error counting stops before this symbol (0: n_sym - 64) */
  int32_t dd_phase;      /* KK: 0, Viterbi-Viterbi carrier phase per block after the DD-LMS; 1, none:
                            the DD-LMS taps track the phase (the paper's short DD-LMS doing clock-
                            and symbol-phase recovery, Sec. 2 second paragraph) */
  int32_t pad2;
} rxo_cfg;

/* Optional outputs: any pointer may be NULL. */
typedef struct rxo_out_s {
  double *field;     /* KK: reconstructed field E (2*L doubles, re/im) before carrier removal */
  double *shifted;   /* KK: (E - mean) * exp(-j 2 pi frac(r n)) (2*L doubles) */
  double *mf;        /* PAM: AGC'd MF output (L); KK: AGC'd decimated MF output (2*(L/2)) */
  double *timing;    /* PAM: timing shift delta_b in samples per 512-sample block (L/512) */
  double *xr;        /* PAM: timing-corrected 2-sps samples (L) */
  double *soft;      /* soft symbols in odd-integer units: PAM nsym, KK 2*nsym (after VV) */
  double *taps;      /* prefix taps w0 as complex pairs (2*ffe_taps) */
  double *phase;     /* KK: unwrapped per-block carrier phase (nsym/128) */
  double *ddz;       /* equaliser outputs before the carrier-phase derotation (PAM nsym, KK 2*nsym):
                        the values the block DD-LMS decides on */
  uint8_t *bits;     /* packed hard decisions, ceil(nsym*bps/8) bytes */
  double mean_re, mean_im;   /* KK: carrier mean; PAM: mean of v */
  double agc, theta0;
  int32_t lag, rot, fallback, pad1;
  int64_t nsym, nbits, counted_syms, sym_errors, counted_bits, bit_errors;
} rxo_out;

#define RXO_FD_EQ_TAPS 203   /* the paper's KK static equaliser length */
#define RXO_FD_PAM_EQ_TAPS 503   /* the paper's PAM static equaliser length */
#define RXO_MLP_IN 31
#define RXO_MLP_H 64
#define RXO_MLP_PARAMS (RXO_MLP_H * RXO_MLP_IN + RXO_MLP_H + RXO_MLP_H * RXO_MLP_H + RXO_MLP_H + RXO_MLP_H + 1)

int rxo_process(const rxo_cfg *cfg, const uint8_t *packed, int64_t n_samples, rxo_out *out);

/* building blocks, exported for the pins */
uint64_t rxo_splitmix64(uint64_t seed, uint64_t k);
void rxo_unpack12(const uint8_t *in, int64_t n, int32_t *codes);
void rxo_fft(double *x, int64_t n, int inverse);
void rxo_rrc_taps(int32_t k, double sps, double beta, double *h);
void rxo_hilbert_taps(int32_t ntaps, double *h);
void rxo_fir_same(const double *x, int64_t n, const double *h, int32_t k, double *y);
void rxo_fir_same_dec2_cplx(const double *x, int64_t n, const double *h, int32_t k, double *y);
void rxo_hilbert_direct(const double *l, int64_t n, const double *h, int32_t ntaps, double *phi);
void rxo_hilbert_os(const double *l, int64_t n, const double *h, int32_t ntaps, int32_t log2n, double *phi);
void rxo_hilbert_fd(const double *l, int64_t n, double *phi);
void rxo_fd_eq_dec2(const double *y, int64_t n, const double *h, int32_t ntaps, double *x);
void rxo_fd_fir(const double *x, int64_t n, const double *h, int32_t ntaps, double *y);
void rxo_fd_delay(const double *x, int64_t n, const double *delta, double *xr);
void rxo_gardner_sums(const double *x, int64_t n, double *c);
void rxo_gardner(const double *x, int64_t n, double *delta);
void rxo_farrow(const double *x, int64_t n, const double *delta, double *xr);
int32_t rxo_decide(double v, int32_t m_axis);
double rxo_downshift_rev(double r, int64_t n);
void rxo_lms(const double *x, int64_t nx, double *w, int32_t k, int64_t pos0, int64_t count,
             const double *ref, int32_t m_axis, int32_t cplx_axis, double mu, const int32_t *force,
             double *z);
void rxo_cma(const double *x, int64_t nx, double *w, int32_t k, int64_t count, double mu, double r2,
             int64_t nvv, double *s4, double *z);
void rxo_vv_phase(const double *s4, int64_t nb, double *phase);
double rxo_round_bf16(double v);
double rxo_round_fp16(double v);
void rxo_mlp_forward(const double *p, const double *x, int64_t nb, int32_t rounding, double *y);
double rxo_mlp_grad(const double *p, const double *x, const double *t, int64_t nb, double *g);
void rxo_adam(double *p, double *m, double *v, const double *g, int64_t n, int64_t step,
              double lr, double b1, double b2, double eps);

#ifdef __cplusplus
}
#endif
#endif

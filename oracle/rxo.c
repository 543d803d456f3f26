/*
 * rxo.c -- FP64 CPU oracle of the GPU-based software-defined receiver
 * (van der Heide et al., "Real-time, Software-Defined, GPU-Based Receiver
 * Field Trial", ECOC 2020).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Plain C99,
 * double precision, one thread, no fast-math.  Each step follows the chain
 * as the paper describes it (Sec. 2 for the two DSP chains, Fig. 1 for the
 * data flow) with the readings, where the paper is silent, that the design
 * notes list.  Every filter is pinned to its plain linear-convolution
 * definition; the overlap-save FFT below is only a faster way to the same
 * numbers and is itself checked against direct convolution.
 */
#include "rxo.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* Reference sequence: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).  */
/* The k-th output of the generator seeded with `seed`, computed       */
/* directly from the counter (state = seed + (k+1) * gamma).           */
/* ------------------------------------------------------------------ */
uint64_t rxo_splitmix64(uint64_t seed, uint64_t k)
{
  uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* 12-bit ADC samples (Sec. 2, first paragraph): two codes per three bytes,
 * little-endian, the first code in the low 12 bits. */
void rxo_unpack12(const uint8_t *in, int64_t n, int32_t *codes)
{
  for (int64_t i = 0; i < n / 2; i++) {
    const uint8_t *b = in + 3 * i;
    codes[2 * i] = (int32_t)b[0] | ((int32_t)(b[1] & 0x0F) << 8);
    codes[2 * i + 1] = (int32_t)(b[1] >> 4) | ((int32_t)b[2] << 4);
  }
}

/* ------------------------------------------------------------------ */
/* Radix-2 FFT (Cooley-Tukey, bit-reversal then butterflies).  x holds  */
/* n complex numbers as re/im pairs; forward kernel exp(-j 2 pi k n/N), */
/* inverse exp(+j ...), no normalisation.  n must be a power of two.   */
/* ------------------------------------------------------------------ */
void rxo_fft(double *xv, int64_t n, int inverse)
{
  cplx *x = (cplx *)xv;
  for (int64_t i = 1, j = 0; i < n; i++) {
    int64_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) { cplx t = x[i]; x[i] = x[j]; x[j] = t; }
  }
  cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)(n > 1 ? n / 2 : 1));
  for (int64_t len = 2; len <= n; len <<= 1) {
    double sgn = inverse ? 1.0 : -1.0;
    for (int64_t k = 0; k < len / 2; k++) {
      double a = sgn * 2.0 * M_PI * (double)k / (double)len;
      tw[k] = cos(a) + I * sin(a);
    }
    for (int64_t i = 0; i < n; i += len)
      for (int64_t k = 0; k < len / 2; k++) {
        cplx u = x[i + k], v = x[i + k + len / 2] * tw[k];
        x[i + k] = u + v;
        x[i + k + len / 2] = u - v;
      }
  }
  free(tw);
}

/* ------------------------------------------------------------------ */
/* Filter designs                                                      */
/* ------------------------------------------------------------------ */

/* Root-raised-cosine matched filter taps: h[i] = rrc((i-(K-1)/2)/sps; beta)
 * in closed form, with its limits at t = 0 and |t| = 1/(4 beta), scaled to
 * unit energy.  (The paper's receivers filter with long static equalisers,
 * Sec. 2; here the matched filter is the RRC of the transmitter, Sec. 3.) */
void rxo_rrc_taps(int32_t k, double sps, double beta, double *h)
{
  double e = 0.0;
  for (int32_t i = 0; i < k; i++) {
    double t = ((double)i - 0.5 * (double)(k - 1)) / sps;
    double v;
    if (fabs(t) < 1e-12) {
      v = 1.0 - beta + 4.0 * beta / M_PI;
    } else if (beta > 0 && fabs(fabs(t) - 1.0 / (4.0 * beta)) < 1e-12) {
      v = beta / sqrt(2.0) * ((1.0 + 2.0 / M_PI) * sin(M_PI / (4.0 * beta)) +
                              (1.0 - 2.0 / M_PI) * cos(M_PI / (4.0 * beta)));
    } else {
      v = (sin(M_PI * t * (1.0 - beta)) + 4.0 * beta * t * cos(M_PI * t * (1.0 + beta))) /
          (M_PI * t * (1.0 - (4.0 * beta * t) * (4.0 * beta * t)));
    }
    h[i] = v;
    e += v * v;
  }
  e = 1.0 / sqrt(e);
  for (int32_t i = 0; i < k; i++) h[i] *= e;
}

/* Finite Hilbert transformer for the Kramers-Kronig phase (Sec. 2, second
 * paragraph, done there with FFTs): ntaps = V+1 taps, index i <-> offset
 * m = i - V/2; h = (2/(pi m)) w(m) for odd m, 0 for even m, with the
 * Blackman window w(m) = 0.42 + 0.5 cos(2 pi m/V) + 0.08 cos(4 pi m/V). */
void rxo_hilbert_taps(int32_t ntaps, double *h)
{
  int32_t v = ntaps - 1;
  for (int32_t i = 0; i < ntaps; i++) {
    int32_t m = i - v / 2;
    if (m % 2 == 0) {
      h[i] = 0.0;
    } else {
      double w = 0.42 + 0.5 * cos(2.0 * M_PI * m / v) + 0.08 * cos(4.0 * M_PI * m / v);
      h[i] = 2.0 / (M_PI * (double)m) * w;
    }
  }
}

/* ------------------------------------------------------------------ */
/* Plain convolutions (the definitions)                                */
/* ------------------------------------------------------------------ */

/* Centred ("same") FIR, zero outside the buffer:
 * y[n] = sum_i h[i] x[n + (K-1)/2 - i]. */
void rxo_fir_same(const double *x, int64_t n, const double *h, int32_t k, double *y)
{
  int32_t c = (k - 1) / 2;
  for (int64_t t = 0; t < n; t++) {
    double acc = 0.0;
    for (int32_t i = 0; i < k; i++) {
      int64_t j = t + c - i;
      if (j >= 0 && j < n) acc += h[i] * x[j];
    }
    y[t] = acc;
  }
}

/* Same FIR on a complex sequence, keeping the even outputs only
 * (decimation to 2 samples per symbol): y[m] = sum_i h[i] x[2m + c - i]. */
void rxo_fir_same_dec2_cplx(const double *xv, int64_t n, const double *h, int32_t k, double *yv)
{
  const cplx *x = (const cplx *)xv;
  cplx *y = (cplx *)yv;
  int32_t c = (k - 1) / 2;
  for (int64_t m = 0; m < n / 2; m++) {
    cplx acc = 0.0;
    for (int32_t i = 0; i < k; i++) {
      int64_t j = 2 * m + c - i;
      if (j >= 0 && j < n) acc += h[i] * x[j];
    }
    y[m] = acc;
  }
}

static inline double edge(const double *l, int64_t n, int64_t j)
{
  return l[j < 0 ? 0 : (j >= n ? n - 1 : j)];
}

/* x[j] inside the buffer, zero outside */
static inline double at(const double *x, int64_t n, int64_t j) { return (j >= 0 && j < n) ? x[j] : 0.0; }

/* Hilbert FIR applied directly, input replicated beyond the buffer edges:
 * phi[t] = sum_m h(m) l[t - m]. */
void rxo_hilbert_direct(const double *l, int64_t n, const double *h, int32_t ntaps, double *phi)
{
  int32_t half = (ntaps - 1) / 2;
  for (int64_t t = 0; t < n; t++) {
    double acc = 0.0;
    for (int32_t i = 0; i < ntaps; i++) {
      if (h[i] == 0.0) continue;
      acc += h[i] * edge(l, n, t - (i - half));
    }
    phi[t] = acc;
  }
}

/* The same convolution by overlap-save with N-point FFTs (hop N - V): each
 * block's circular convolution equals the linear one on its N - V central
 * outputs. */
void rxo_hilbert_os(const double *l, int64_t n, const double *h, int32_t ntaps, int32_t log2n, double *phi)
{
  int64_t big = (int64_t)1 << log2n;
  int32_t v = ntaps - 1, half = v / 2;
  int64_t hop = big - v;
  double *hf = (double *)calloc((size_t)(2 * big), sizeof(double));
  double *buf = (double *)malloc(sizeof(double) * (size_t)(2 * big));
  for (int32_t i = 0; i < ntaps; i++) {
    int64_t p = ((int64_t)(i - half) % big + big) % big;
    hf[2 * p] += h[i];
  }
  rxo_fft(hf, big, 0);
  for (int64_t n0 = 0; n0 < n; n0 += hop) {
    for (int64_t p = 0; p < big; p++) {
      buf[2 * p] = edge(l, n, n0 - half + p);
      buf[2 * p + 1] = 0.0;
    }
    rxo_fft(buf, big, 0);
    for (int64_t p = 0; p < big; p++) {
      cplx a = buf[2 * p] + I * buf[2 * p + 1];
      cplx b = hf[2 * p] + I * hf[2 * p + 1];
      cplx r = a * b;
      buf[2 * p] = creal(r);
      buf[2 * p + 1] = cimag(r);
    }
    rxo_fft(buf, big, 1);
    for (int64_t q = 0; q < hop && n0 + q < n; q++) phi[n0 + q] = buf[2 * (half + q)] / (double)big;
  }
  free(hf);
  free(buf);
}

/* The paper's frequency-domain forms (Sec. 2, first and second paragraphs:
 * 1024-point transforms over blocks that advance by 512 samples, "100 %
 * overlap", 8192 blocks per 2^22-sample buffer).  Block b covers samples
 * 512 b - 256 .. 512 b + 767 and yields the 512 samples at its centre,
 * 512 b .. 512 b + 511. */
#define FD_N 1024
#define FD_HOP 512
#define FD_GUARD 256

/* Hilbert transform by the block-circular -j sgn(k) on each block's
 * 1024-point spectrum (sgn = 0 at DC and at N/2); samples before the buffer
 * repeat its first one and samples after it its last one. */
void rxo_hilbert_fd(const double *l, int64_t n, double *phi)
{
  cplx *buf = (cplx *)malloc(sizeof(cplx) * FD_N);
  for (int64_t b = 0; b * FD_HOP < n; b++) {
    const int64_t t0 = b * FD_HOP - FD_GUARD;
    for (int t = 0; t < FD_N; t++) buf[t] = edge(l, n, t0 + t);
    rxo_fft((double *)buf, FD_N, 0);
    for (int k = 0; k < FD_N; k++) {
      const double sg = (k == 0 || k == FD_N / 2) ? 0.0 : (k < FD_N / 2 ? 1.0 : -1.0);
      buf[k] *= -I * sg;
    }
    rxo_fft((double *)buf, FD_N, 1);
    for (int u = 0; u < FD_HOP && b * FD_HOP + u < n; u++) phi[b * FD_HOP + u] = creal(buf[FD_GUARD + u]) / FD_N;
  }
  free(buf);
}

/* Static equaliser and decimation to 2 samples per symbol in the frequency
 * domain: each block's 1024-point spectrum (samples outside the buffer are
 * zero) times the response of the ntaps-tap filter h (centred: tap i at
 * offset i - (ntaps - 1) / 2, taken circularly), then the 512 bins of
 * |f| < fs / 4 (k < 256 and k >= 768) through a 512-point inverse transform
 * (scaled 1 / 1024), whose outputs are the filtered block at every second
 * sample; the block's central 256 outputs are kept.  y, x: complex, n and
 * n / 2 values. */
void rxo_fd_eq_dec2(const double *yv, int64_t n, const double *h, int32_t ntaps, double *xv)
{
  const cplx *y = (const cplx *)yv;
  cplx *x = (cplx *)xv;
  cplx *buf = (cplx *)malloc(sizeof(cplx) * FD_N), *hf = (cplx *)calloc(FD_N, sizeof(cplx));
  cplx *z = (cplx *)malloc(sizeof(cplx) * FD_N / 2);
  const int32_t c = (ntaps - 1) / 2;
  for (int32_t i = 0; i < ntaps; i++) hf[((i - c) % FD_N + FD_N) % FD_N] += h[i];
  rxo_fft((double *)hf, FD_N, 0);
  for (int64_t b = 0; b * FD_HOP < n; b++) {
    const int64_t t0 = b * FD_HOP - FD_GUARD;
    for (int t = 0; t < FD_N; t++) buf[t] = (t0 + t >= 0 && t0 + t < n) ? y[t0 + t] : 0.0;
    rxo_fft((double *)buf, FD_N, 0);
    for (int k = 0; k < FD_N / 2; k++) {
      const int kk = k < FD_N / 4 ? k : k + FD_N / 2;
      z[k] = buf[kk] * hf[kk];
    }
    rxo_fft((double *)z, FD_N / 2, 1);
    for (int u = 0; u < FD_HOP / 2 && b * FD_HOP + 2 * u < n; u++)
      x[b * (FD_HOP / 2) + u] = z[FD_GUARD / 2 + u] / FD_N;
  }
  free(buf); free(hf); free(z);
}

/* A real FIR in the frequency domain on the same blocks: each block's
 * spectrum (samples outside the buffer are zero) times the response of the
 * centred ntaps-tap filter, back, central 512 samples kept.  For ntaps up to
 * 2 * 256 + 1 no central output wraps around the block, so this is the
 * "same" convolution with zeros outside the buffer, by another route. */
void rxo_fd_fir(const double *x, int64_t n, const double *h, int32_t ntaps, double *y)
{
  cplx *buf = (cplx *)malloc(sizeof(cplx) * FD_N), *hf = (cplx *)calloc(FD_N, sizeof(cplx));
  const int32_t c = (ntaps - 1) / 2;
  for (int32_t i = 0; i < ntaps; i++) hf[((i - c) % FD_N + FD_N) % FD_N] += h[i];
  rxo_fft((double *)hf, FD_N, 0);
  for (int64_t b = 0; b * FD_HOP < n; b++) {
    const int64_t t0 = b * FD_HOP - FD_GUARD;
    for (int t = 0; t < FD_N; t++) buf[t] = at(x, n, t0 + t);
    rxo_fft((double *)buf, FD_N, 0);
    for (int k = 0; k < FD_N; k++) buf[k] *= hf[k];
    rxo_fft((double *)buf, FD_N, 1);
    for (int u = 0; u < FD_HOP && b * FD_HOP + u < n; u++) y[b * FD_HOP + u] = creal(buf[FD_GUARD + u]) / FD_N;
  }
  free(buf); free(hf);
}

/* Timing correction in the frequency domain: block b's central samples are
 * the block resampled at t + delta[b] (delta in samples, one per 512-sample
 * block, as rxo_gardner gives it), i.e. its spectrum times exp(+j 2 pi k d /
 * N) for the signed bin index k in (-N/2, N/2) and cos(pi d) at N/2 (the
 * real part of either sign, so the result stays real). */
void rxo_fd_delay(const double *x, int64_t n, const double *delta, double *xr)
{
  cplx *buf = (cplx *)malloc(sizeof(cplx) * FD_N);
  for (int64_t b = 0; b * FD_HOP < n; b++) {
    const int64_t t0 = b * FD_HOP - FD_GUARD;
    const double d = delta[b];
    for (int t = 0; t < FD_N; t++) buf[t] = at(x, n, t0 + t);
    rxo_fft((double *)buf, FD_N, 0);
    for (int k = 0; k < FD_N; k++) {
      if (k == FD_N / 2) buf[k] *= cos(M_PI * d);
      else buf[k] *= cexp(2.0 * M_PI * I * (double)(k < FD_N / 2 ? k : k - FD_N) * d / FD_N);
    }
    rxo_fft((double *)buf, FD_N, 1);
    for (int u = 0; u < FD_HOP && b * FD_HOP + u < n; u++) xr[b * FD_HOP + u] = creal(buf[FD_GUARD + u]) / FD_N;
  }
  free(buf);
}

/* ------------------------------------------------------------------ */
/* Rounding to the narrow operand formats of the precision form          */
/* (round to nearest, ties to even).                                     */
/* ------------------------------------------------------------------ */
static double round_bits(double v, int mant_bits, int min_exp)
{
  if (v == 0.0 || !isfinite(v)) return v;
  int e;
  frexp(v, &e);                 /* v = f * 2^e, 0.5 <= |f| < 1 */
  if (e - 1 < min_exp) e = min_exp + 1;
  double scale = ldexp(1.0, mant_bits - e);
  return nearbyint(v * scale) / scale;
}
double rxo_round_bf16(double v) { return round_bits(v, 8, -126); }
double rxo_round_fp16(double v) { return round_bits(v, 11, -14); }
static double rnd(int mode, double v)
{
  return mode == 1 ? rxo_round_bf16(v) : (mode == 2 ? rxo_round_fp16(v) : v);
}
static cplx rndc(int mode, cplx v) { return rnd(mode, creal(v)) + I * rnd(mode, cimag(v)); }

/* ------------------------------------------------------------------ */
/* Decisions and Gray demapping (Sec. 2, first and second paragraphs). */
/* Levels 2i-(M-1) per real axis, thresholds at the even integers, an    */
/* exact tie goes to the higher level; bits = i xor (i >> 1), MSB first. */
/* ------------------------------------------------------------------ */
int32_t rxo_decide(double v, int32_t m)
{
  double f = floor((v + (double)m) / 2.0);
  if (f < 0) f = 0;
  if (f > m - 1) f = m - 1;
  return (int32_t)f;
}

static int bps_of(int fmt) { return fmt == 1 ? 1 : fmt == 2 ? 2 : fmt == 3 ? 3 : fmt == 4 ? 2 : 4; }
static int is_kk(int fmt) { return fmt >= RXO_KK_QPSK; }
static int axis_levels(int fmt) { return fmt == 1 ? 2 : fmt == 2 ? 4 : fmt == 3 ? 8 : fmt == 4 ? 2 : 4; }

static uint32_t gray(uint32_t i) { return i ^ (i >> 1); }
static uint32_t gray_inv(uint32_t g)
{
  uint32_t i = g;
  for (uint32_t s = g >> 1; s; s >>= 1) i ^= s;
  return i;
}

/* Transmitted symbol k of the reference sequence, in odd-integer units. */
static cplx ref_symbol(int fmt, uint64_t seed, int64_t k)
{
  int bps = bps_of(fmt);
  uint32_t b = (uint32_t)(rxo_splitmix64(seed, (uint64_t)k) >> (64 - bps));
  if (is_kk(fmt)) {
    int half = bps / 2, m = 1 << half;
    uint32_t bi = b >> half, bq = b & (uint32_t)(m - 1);
    return (double)(2 * (int)gray_inv(bi) - (m - 1)) + I * (double)(2 * (int)gray_inv(bq) - (m - 1));
  }
  int m = 1 << bps;
  return (double)(2 * (int)gray_inv(b) - (m - 1));
}

/* Hard decision of a soft symbol, as a point of the constellation. */
static cplx decide_point(int fmt, cplx z)
{
  int m = axis_levels(fmt);
  double re = 2.0 * rxo_decide(creal(z), m) - (m - 1);
  if (!is_kk(fmt)) return re;
  return re + I * (2.0 * rxo_decide(cimag(z), m) - (m - 1));
}

static uint32_t symbol_bits(int fmt, cplx z)
{
  int m = axis_levels(fmt);
  uint32_t gi = gray((uint32_t)rxo_decide(creal(z), m));
  if (!is_kk(fmt)) return gi;
  int half = bps_of(fmt) / 2;
  return (gi << half) | gray((uint32_t)rxo_decide(cimag(z), m));
}

/* ------------------------------------------------------------------ */
/* Timing recovery of the PAM chain (Sec. 2, first paragraph: blockwise  */
/* clock-phase estimation, unwrapping, clock recovery), as feed-forward  */
/* Gardner estimation per 256-symbol block.                              */
/* ------------------------------------------------------------------ */

/* Detector sums per 512-sample block (256 symbols): C_b = G0_b + j G1_b,
 * G0 the Gardner detector on the symbol-spaced samples, G1 the same detector
 * a quarter symbol (half a sample) later, its samples taken by cubic Lagrange
 * interpolation at mu = 1/2. */
void rxo_gardner_sums(const double *x, int64_t n, double *cv)
{
  const int64_t nb = n / 512;
  cplx *c = (cplx *)cv;
  for (int64_t b = 0; b < nb; b++) {
    double g0 = 0.0, g1 = 0.0;
    for (int64_t k = b * 256; k < (b + 1) * 256; k++) {
      int64_t s = 2 * k;
      g0 += at(x, n, s + 1) * (at(x, n, s) - at(x, n, s + 2));
      double h0 = (-at(x, n, s - 1) + 9.0 * at(x, n, s) + 9.0 * at(x, n, s + 1) - at(x, n, s + 2)) / 16.0;
      double h1 = (-at(x, n, s) + 9.0 * at(x, n, s + 1) + 9.0 * at(x, n, s + 2) - at(x, n, s + 3)) / 16.0;
      double h2 = (-at(x, n, s + 1) + 9.0 * at(x, n, s + 2) + 9.0 * at(x, n, s + 3) - at(x, n, s + 4)) / 16.0;
      g1 += h1 * (h0 - h2);
    }
    c[b] = g0 + I * g1;
  }
}

/* Feed-forward timing estimate per block: the sums averaged over blocks
 * b-16..b+16 (clipped at the ends), their angle, unwrapped across blocks,
 * as a shift in samples.  The half-sample interpolator has the gain
 * (18 cos(pi/4) - 2 cos(3 pi/4)) / 16 = 5 / (4 sqrt 2) at half the symbol
 * rate, where the detector's timing information sits, and G1 is a product
 * of two interpolated samples: it is scaled back by the inverse squared
 * gain, 32 / 25, so that G0 and G1 are a quadrature pair of equal weight. */
void rxo_gardner(const double *x, int64_t n, double *delta)
{
  const int64_t nb = n / 512, win = 16;
  cplx *c = (cplx *)malloc(sizeof(cplx) * (size_t)(nb > 0 ? nb : 1));
  rxo_gardner_sums(x, n, (double *)c);
  double prev_raw = 0.0, acc = 0.0;
  for (int64_t b = 0; b < nb; b++) {
    cplx s = 0.0;
    int64_t lo = b - win < 0 ? 0 : b - win, hi = b + win >= nb ? nb - 1 : b + win;
    for (int64_t j = lo; j <= hi; j++) s += c[j];
    double raw = atan2(cimag(s) * (32.0 / 25.0), creal(s));
    if (b == 0) {
      acc = raw;
    } else {
      double d = raw - prev_raw;
      acc += d - 2.0 * M_PI * floor(d / (2.0 * M_PI) + 0.5);
    }
    prev_raw = raw;
    delta[b] = 0.5 + acc / M_PI;      /* shift in samples (one symbol = 2) */
  }
  free(c);
}

/* Cubic-Lagrange (Farrow) interpolation onto the recovered grid:
 * xr[t] = x(t + delta_b) for t in block b. */
void rxo_farrow(const double *x, int64_t n, const double *delta, double *xr)
{
  for (int64_t t = 0; t < n; t++) {
    double d = delta[t / 512];
    double fl = floor(d), mu = d - fl;
    int64_t i0 = t + (int64_t)fl;
    double lm1 = -mu * (mu - 1.0) * (mu - 2.0) / 6.0;
    double l0 = (mu + 1.0) * (mu - 1.0) * (mu - 2.0) / 2.0;
    double l1 = -(mu + 1.0) * mu * (mu - 2.0) / 2.0;
    double l2 = (mu + 1.0) * mu * (mu - 1.0) / 6.0;
    xr[t] = lm1 * at(x, n, i0 - 1) + l0 * at(x, n, i0) + l1 * at(x, n, i0 + 1) + l2 * at(x, n, i0 + 2);
  }
}

/* ------------------------------------------------------------------ */
/* Small MLP equaliser: 31 -> 64 ReLU -> 64 ReLU -> 1.                  */
/* Parameters packed W1[64][31], b1, W2[64][64], b2, W3[64], b3.        */
/* rounding 1/2: the operands of all three layers (inputs, weights,     */
/* hidden activations) rounded to BF16/FP16, products summed in FP64,   */
/* biases exact: inference on narrow matrix operands with a wide        */
/* accumulator throughout.                                              */
/* ------------------------------------------------------------------ */
#define H RXO_MLP_H
#define NI RXO_MLP_IN
static void mlp_one(const double *p, const double *x, int rm, double *h1, double *h2, double *y)
{
  const double *w1 = p, *b1 = w1 + H * NI, *w2 = b1 + H, *b2 = w2 + H * H, *w3 = b2 + H, *b3 = w3 + H;
  for (int o = 0; o < H; o++) {
    double a = 0.0;
    for (int i = 0; i < NI; i++) a += rnd(rm, w1[o * NI + i]) * rnd(rm, x[i]);
    a += b1[o];
    h1[o] = a > 0.0 ? a : 0.0;
  }
  for (int o = 0; o < H; o++) {
    double a = 0.0;
    for (int i = 0; i < H; i++) a += rnd(rm, w2[o * H + i]) * rnd(rm, h1[i]);
    a += b2[o];
    h2[o] = a > 0.0 ? a : 0.0;
  }
  double a = b3[0];
  for (int i = 0; i < H; i++) a += rnd(rm, w3[i]) * rnd(rm, h2[i]);
  *y = a;
}

void rxo_mlp_forward(const double *p, const double *x, int64_t nb, int32_t rounding, double *y)
{
  double h1[H], h2[H];
  for (int64_t s = 0; s < nb; s++) mlp_one(p, x + s * NI, rounding, h1, h2, y + s);
}

/* Mean-squared-error loss (1/B) sum (y - t)^2 of a minibatch and its
 * gradient with respect to every parameter (backpropagation). */
double rxo_mlp_grad(const double *p, const double *x, const double *t, int64_t nb, double *g)
{
  const double *w2 = p + H * NI + H, *w3 = w2 + H * H + H;
  double *gw1 = g, *gb1 = gw1 + H * NI, *gw2 = gb1 + H, *gb2 = gw2 + H * H, *gw3 = gb2 + H, *gb3 = gw3 + H;
  memset(g, 0, sizeof(double) * RXO_MLP_PARAMS);
  double loss = 0.0, h1[H], h2[H], d2[H], d1[H], y;
  for (int64_t s = 0; s < nb; s++) {
    const double *xs = x + s * NI;
    mlp_one(p, xs, 0, h1, h2, &y);
    double r = y - t[s];
    loss += r * r;
    double dy = 2.0 * r / (double)nb;
    gb3[0] += dy;
    for (int i = 0; i < H; i++) {
      gw3[i] += dy * h2[i];
      d2[i] = h2[i] > 0.0 ? dy * w3[i] : 0.0;
    }
    for (int o = 0; o < H; o++) {
      gb2[o] += d2[o];
      for (int i = 0; i < H; i++) gw2[o * H + i] += d2[o] * h1[i];
    }
    for (int i = 0; i < H; i++) {
      double a = 0.0;
      for (int o = 0; o < H; o++) a += w2[o * H + i] * d2[o];
      d1[i] = h1[i] > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < H; o++) {
      gb1[o] += d1[o];
      for (int i = 0; i < NI; i++) gw1[o * NI + i] += d1[o] * xs[i];
    }
  }
  return loss / (double)nb;
}

/* Adam (Kingma & Ba, ICLR 2015), step counted from 1. */
void rxo_adam(double *p, double *m, double *v, const double *g, int64_t n, int64_t step,
              double lr, double b1, double b2, double eps)
{
  double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
  for (int64_t i = 0; i < n; i++) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}
#undef H
#undef NI

/* ------------------------------------------------------------------ */
/* T/2-spaced FFE (one sample pair per symbol).  Output for reference   */
/* symbol k uses x[2(k+s) + c - i], i = 0..K-1, zero outside.           */
/* ------------------------------------------------------------------ */
static inline cplx xat(const cplx *x, int64_t n, int64_t j) { return (j >= 0 && j < n) ? x[j] : 0.0; }

static cplx ffe_out(const cplx *x, int64_t n, const cplx *w, int k, int64_t pos)
{
  int c = (k - 1) / 2;
  cplx z = 0.0;
  for (int i = 0; i < k; i++) z += w[i] * xat(x, n, pos + c - i);
  return z;
}

static void ffe_update(const cplx *x, int64_t n, cplx *w, int k, int64_t pos, cplx step)
{
  int c = (k - 1) / 2;
  for (int i = 0; i < k; i++) w[i] += step * conj(xat(x, n, pos + c - i));
}

static double level(int32_t i, int32_t m) { return 2.0 * (double)i - (double)(m - 1); }

/* LMS adaptation of the FFE over `count` symbols (Sec. 2: the PAM chain's
 * LMS FFE, the KK chain's DD-LMS): for symbol j the output
 * z_j = sum_i w_i x[pos0 + 2j + c - i] is formed first, then
 * w_i += mu (d_j - z_j) conj(x[pos0 + 2j + c - i]).  d_j is ref[j] when a
 * reference is given (training on known symbols), else the decision of z_j
 * (m_axis levels per real axis; both axes when cplx_axis).  force[j] >= 0,
 * if given, replaces decision j by the level with that index (i m + q for
 * QAM): test instrumentation that follows another implementation's choice
 * at a symbol lying on a threshold. */
void rxo_lms(const double *xv, int64_t nx, double *wv, int32_t k, int64_t pos0, int64_t count,
             const double *refv, int32_t m_axis, int32_t cplx_axis, double mu, const int32_t *force,
             double *zv)
{
  const cplx *x = (const cplx *)xv, *ref = (const cplx *)refv;
  cplx *w = (cplx *)wv, *zo = (cplx *)zv;
  for (int64_t j = 0; j < count; j++) {
    const int64_t pos = pos0 + 2 * j;
    cplx z = ffe_out(x, nx, w, k, pos), d;
    if (zo) zo[j] = z;
    if (ref) {
      d = ref[j];
    } else if (force && force[j] >= 0) {
      d = cplx_axis ? level(force[j] / m_axis, m_axis) + I * level(force[j] % m_axis, m_axis)
                    : level(force[j], m_axis);
    } else {
      d = level(rxo_decide(creal(z), m_axis), m_axis);
      if (cplx_axis) d += I * level(rxo_decide(cimag(z), m_axis), m_axis);
    }
    ffe_update(x, nx, w, k, pos, mu * (d - z));
  }
}

/* Constant-modulus adaptation from sample 0 over `count` symbols: z_j as
 * above (pos0 = 0), then w_i += mu z_j (r2 - |z_j|^2) conj(x[2j + c - i]).
 * s4 (re, im) receives the sum of z_j^4 over the last nvv outputs (the
 * static Viterbi-Viterbi phase estimate); z (optional) the outputs. */
void rxo_cma(const double *xv, int64_t nx, double *wv, int32_t k, int64_t count, double mu, double r2,
             int64_t nvv, double *s4v, double *zv)
{
  const cplx *x = (const cplx *)xv;
  cplx *w = (cplx *)wv, *zo = (cplx *)zv, s4 = 0.0;
  for (int64_t j = 0; j < count; j++) {
    cplx z = ffe_out(x, nx, w, k, 2 * j);
    if (zo) zo[j] = z;
    if (j >= count - nvv) s4 += z * z * z * z;
    double mag = creal(z) * creal(z) + cimag(z) * cimag(z);
    ffe_update(x, nx, w, k, 2 * j, mu * z * (r2 - mag));
  }
  s4v[0] = creal(s4);
  s4v[1] = cimag(s4);
}

/* Viterbi-Viterbi carrier phase per block from the blocks' sums of z^4:
 * theta_b = 1/4 arg(-(S_{b-1} + S_b + S_{b+1})) (neighbours beyond the ends
 * left out; E[a^4] < 0 for QPSK and 16QAM), unwrapped across blocks in
 * multiples of pi/2, the symmetry of the constellation. */
void rxo_vv_phase(const double *s4v, int64_t nb, double *phase)
{
  const cplx *s4 = (const cplx *)s4v;
  double prev = 0.0, th = 0.0;
  for (int64_t b = 0; b < nb; b++) {
    cplx a = s4[b] + (b > 0 ? s4[b - 1] : 0.0) + (b + 1 < nb ? s4[b + 1] : 0.0);
    double raw = 0.25 * carg(-a);
    if (b == 0) {
      th = raw;
    } else {
      double d = raw - prev;
      th += d - (M_PI / 2.0) * floor(d / (M_PI / 2.0) + 0.5);
    }
    prev = raw;
    phase[b] = th;
  }
}

/* Downshift phase of sample n in revolutions, frac(r n), in FP64 (the
 * frequency shift of the KK chain, Fig. 1d). */
double rxo_downshift_rev(double r, int64_t n)
{
  double u = r * (double)n;
  return u - floor(u);
}

/* Joint delay / rotation search on the known prefix: maximise
 * |sum_k z(k+s) conj(a_k)| over s in [-64, 64] (ties: smallest |s|, then
 * the negative one); rotation j^q with q = round(-arg(C)/(pi/2)) (KK only). */
static void sync_search(int fmt, const cplx *x, int64_t n, const cplx *w, int k, int p,
                        const cplx *a, int32_t *lag, int32_t *rot)
{
  const int R = 64;
  cplx *z = (cplx *)malloc(sizeof(cplx) * (size_t)(p + 2 * R));
  for (int j = -R; j < p + R; j++) z[j + R] = ffe_out(x, n, w, k, 2 * (int64_t)j);
  double best = -INFINITY;
  cplx bestc = 0.0;
  int bests = 0;
  for (int t = 0; t <= 2 * R; t++) {
    int s = (t == 0) ? 0 : ((t & 1) ? -((t + 1) / 2) : t / 2);
    cplx c = 0.0;
    for (int j = 0; j < p; j++) c += z[j + s + R] * conj(a[j]);
    double score = is_kk(fmt) ? cabs(c) : creal(c);
    if (score > best) { best = score; bests = s; bestc = c; }
  }
  *lag = bests;
  *rot = 0;
  if (is_kk(fmt)) {
    long q = lround(-carg(bestc) / (M_PI / 2.0));
    *rot = (int32_t)(((q % 4) + 4) % 4);
  }
  free(z);
}

static const cplx jpow[4] = {1.0, I, -1.0, -I};

/* ------------------------------------------------------------------ */
/* The two chains                                                        */
/* ------------------------------------------------------------------ */
int rxo_process(const rxo_cfg *cfg, const uint8_t *packed, int64_t n, rxo_out *o)
{
  const int fmt = cfg->fmt;
  if (fmt < 1 || fmt > 5 || n <= 0 || n % 1024) return -1;
  const int kk = is_kk(fmt), bps = bps_of(fmt), sps = kk ? 4 : 2, m = axis_levels(fmt);
  const int64_t nsym = n / sps, nd = n / 2;
  const int K = cfg->ffe_taps, c = (K - 1) / 2, P = cfg->prefix, G = 64;
  const int blk = kk ? 128 : 256;
  const int rm = cfg->rounding;
  const rxo_out *fz = cfg->frozen;
  if (P + 2 * G >= nsym || K < 1 || (K % 2 == 0 && K != 4) || cfg->mf_taps % 2 == 0) return -1;
  if (cfg->dd_phase && !kk) return -1;
  if (cfg->equalizer == 1 && (kk || !cfg->mlp)) return -1;
  if (cfg->front == 1 && (rm || fz || cfg->equalizer == 1)) return -1;   /* the FD front end: FP64, one buffer, LMS */

  int32_t *code = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  rxo_unpack12(packed, n, code);
  double *hm = (double *)malloc(sizeof(double) * (size_t)cfg->mf_taps);
  rxo_rrc_taps(cfg->mf_taps, (double)sps, cfg->rolloff, hm);

  cplx *x = (cplx *)malloc(sizeof(cplx) * (size_t)nd * (kk ? 1 : 2)); /* FFE input (2 sps) */
  int64_t nx;
  o->nsym = nsym;
  o->fallback = 0;

  if (kk) {
    /* --- Kramers-Kronig front end (Sec. 2, second paragraph; Fig. 1d) --- */
    double *ell = (double *)malloc(sizeof(double) * (size_t)n);
    double *phi = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t t = 0; t < n; t++) ell[t] = 0.5 * log((double)code[t] + 0.5);
    double *hh = (double *)malloc(sizeof(double) * (size_t)cfg->hilbert_taps);
    rxo_hilbert_taps(cfg->hilbert_taps, hh);
    if (cfg->front == 1) rxo_hilbert_fd(ell, n, phi);
    else rxo_hilbert_os(ell, n, hh, cfg->hilbert_taps, cfg->os_log2, phi);
    const double sg = cfg->fc_over_fs >= 0 ? 1.0 : -1.0;
    cplx *e = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx mean = 0.0;
    for (int64_t t = 0; t < n; t++) {
      e[t] = sqrt((double)code[t] + 0.5) * cexp(I * sg * phi[t]);
      mean += e[t];
    }
    mean /= (double)n;
    if (fz) mean = fz->mean_re + I * fz->mean_im;   /* a stream's carrier from its first buffer */
    if (o->field) memcpy(o->field, e, sizeof(cplx) * (size_t)n);
    /* carrier removal and downshift, the phase frac(r t) kept in FP64 */
    cplx *y = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    for (int64_t t = 0; t < n; t++)
      y[t] = (e[t] - mean) * cexp(-2.0 * M_PI * I * rxo_downshift_rev(cfg->fc_over_fs, t));
    if (o->shifted) memcpy(o->shifted, y, sizeof(cplx) * (size_t)n);
    if (rm) {
      /* precision form: the matched filter's operands, the carrier-free
       * downshifted field and the taps, rounded to the narrow type; the
       * accumulation stays exact */
      for (int64_t t = 0; t < n; t++) y[t] = rndc(rm, y[t]);
      for (int i = 0; i < cfg->mf_taps; i++) hm[i] = rnd(rm, hm[i]);
    }
    if (cfg->front == 1) {
      /* the paper's static equaliser: 203 taps on the 1024-point blocks,
       * here the matched RRC of the same roll-off (its link-specific part
       * is the identity for a back-to-back link) */
      double heq[RXO_FD_EQ_TAPS];
      rxo_rrc_taps(RXO_FD_EQ_TAPS, (double)sps, cfg->rolloff, heq);
      rxo_fd_eq_dec2((double *)y, n, heq, RXO_FD_EQ_TAPS, (double *)x);
    } else {
      rxo_fir_same_dec2_cplx((double *)y, n, hm, cfg->mf_taps, (double *)x);
    }
    nx = nd;
    o->mean_re = creal(mean);
    o->mean_im = cimag(mean);
    free(ell); free(phi); free(hh); free(e); free(y);
  } else {
    /* --- PAM front end (Sec. 2, first paragraph): DC removal, MF --- */
    double s = 0.0;
    for (int64_t t = 0; t < n; t++) s += (double)code[t];
    double mv = fz ? fz->mean_re : s / (double)n + 0.5;
    double *x0 = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t t = 0; t < n; t++) x0[t] = (double)code[t] + 0.5 - mv;
    if (cfg->front == 1) {
      /* the paper's 503-tap static equaliser on the 1024-point blocks (Sec. 2,
       * first paragraph), here the matched RRC of the same roll-off */
      double heq[RXO_FD_PAM_EQ_TAPS];
      rxo_rrc_taps(RXO_FD_PAM_EQ_TAPS, (double)sps, cfg->rolloff, heq);
      rxo_fd_fir(x0, n, heq, RXO_FD_PAM_EQ_TAPS, y);
    } else {
      rxo_fir_same(x0, n, hm, cfg->mf_taps, y);
    }
    o->mean_re = mv;
    o->mean_im = 0.0;
    for (int64_t t = 0; t < n; t++) x[t] = y[t];
    nx = n;
    free(x0); free(y);
  }

  /* --- AGC: unit mean power --- */
  double pw = 0.0;
  for (int64_t t = 0; t < nx; t++) pw += creal(x[t]) * creal(x[t]) + cimag(x[t]) * cimag(x[t]);
  double g = fz ? fz->agc : 1.0 / sqrt(pw / (double)nx);
  for (int64_t t = 0; t < nx; t++) x[t] *= g;
  o->agc = g;
  if (o->mf) {
    for (int64_t t = 0; t < nx; t++) {
      if (kk) { o->mf[2 * t] = creal(x[t]); o->mf[2 * t + 1] = cimag(x[t]); }
      else o->mf[t] = creal(x[t]);
    }
  }

  if (!kk) {
    /* --- timing: Gardner estimate per block, unwrap, Farrow --- */
    double *xs = (double *)malloc(sizeof(double) * (size_t)n);
    double *xr = (double *)malloc(sizeof(double) * (size_t)n);
    double *dl = (double *)malloc(sizeof(double) * (size_t)(n / 512));
    for (int64_t t = 0; t < n; t++) xs[t] = creal(x[t]);
    rxo_gardner(xs, n, dl);
    if (cfg->front == 1) rxo_fd_delay(xs, n, dl, xr);   /* FD clock recovery (Sec. 2, first paragraph) */
    else rxo_farrow(xs, n, dl, xr);
    if (o->timing) memcpy(o->timing, dl, sizeof(double) * (size_t)(n / 512));
    if (o->xr) memcpy(o->xr, xr, sizeof(double) * (size_t)n);
    for (int64_t t = 0; t < n; t++) x[t] = xr[t];
    free(xs); free(xr); free(dl);
  }

  /* --- prefix: (KK) CMA + static VV phase; sync; data-aided LMS --- */
  const double ea2 = (double)(m * m - 1) / 3.0 * (kk ? 2.0 : 1.0);
  cplx *ref = (cplx *)malloc(sizeof(cplx) * (size_t)P);
  for (int k = 0; k < P; k++) ref[k] = ref_symbol(fmt, cfg->seed, k);
  cplx *w = (cplx *)calloc((size_t)K, sizeof(cplx));
  o->theta0 = 0.0;
  if (fz) {
    /* a stream after its first buffer: the acquisition's delay, rotation
     * and prefix taps (the known prefix is only at the stream's start) */
    o->theta0 = fz->theta0;
    o->lag = fz->lag;
    o->rot = fz->rot;
    for (int i = 0; i < K; i++) w[i] = fz->taps[2 * i] + I * fz->taps[2 * i + 1];
  } else if (kk) {
    const double r2 = fmt == RXO_KK_16QAM ? 1.32 : 1.0;
    double s4[2];
    w[c] = 1.0;
    rxo_cma((double *)x, nx, (double *)w, K, P, cfg->mu_cma, r2, 2048, s4, NULL);
    double th = 0.25 * carg(-(s4[0] + I * s4[1]));
    o->theta0 = th;
    cplx rotv = sqrt(ea2) * cexp(-I * th);
    for (int i = 0; i < K; i++) w[i] *= rotv;
  } else {
    w[c] = sqrt(ea2);
  }
  if (!fz) {
    sync_search(fmt, x, nx, w, K, P, ref, &o->lag, &o->rot);
    for (int i = 0; i < K; i++) w[i] *= jpow[o->rot];
    rxo_lms((double *)x, nx, (double *)w, K, 2 * (int64_t)o->lag, P, (double *)ref, m, kk, cfg->mu, NULL, NULL);
  }
  const int64_t sh2 = 2 * (int64_t)o->lag;
  if (o->taps)
    for (int i = 0; i < K; i++) { o->taps[2 * i] = creal(w[i]); o->taps[2 * i + 1] = cimag(w[i]); }

  /* --- equaliser over the whole buffer --- */
  cplx *soft = (cplx *)malloc(sizeof(cplx) * (size_t)nsym);
  int use_mlp = cfg->equalizer == 1;
  if (use_mlp) {
    /* MLP over 31-sample windows centred on each symbol sample; LMS stays
     * the fallback when it makes more errors on the known prefix. */
    double win[RXO_MLP_IN], yv;
    int64_t err_mlp = 0, err_lms = 0;
    for (int64_t k = 0; k < nsym; k++) {
      for (int i = 0; i < RXO_MLP_IN; i++) win[i] = creal(xat(x, nx, sh2 + 2 * k - 15 + i));
      rxo_mlp_forward(cfg->mlp, win, 1, rm, &yv);
      soft[k] = yv;
    }
    for (int64_t k = G; k < P; k++) {
      cplx a = ref[k];
      err_mlp += creal(decide_point(fmt, soft[k])) != creal(a);
      err_lms += creal(decide_point(fmt, ffe_out(x, nx, w, K, sh2 + 2 * k))) != creal(a);
    }
    if (fz ? fz->fallback : err_mlp > err_lms) { use_mlp = 0; o->fallback = 1; }
  }
  if (!use_mlp) {
    cplx *wr = (cplx *)malloc(sizeof(cplx) * (size_t)K);
    cplx *xq = NULL;
    if (cfg->form == 1 && rm) {
      xq = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
      for (int64_t t = 0; t < nx; t++) xq[t] = rndc(rm, x[t]);
    }
    for (int64_t b = 0; b < nsym / blk; b++) {
      for (int i = 0; i < K; i++) wr[i] = (cfg->form == 1) ? rndc(rm, w[i]) : w[i];
      if (cfg->form == 1) {   /* frozen taps: a plain FIR */
        for (int64_t k = b * blk; k < (b + 1) * blk; k++) soft[k] = ffe_out(xq ? xq : x, nx, wr, K, sh2 + 2 * k);
      } else {                /* block DD-LMS from the prefix taps */
        rxo_lms((double *)x, nx, (double *)wr, K, sh2 + 2 * b * blk, blk, NULL, m, kk, cfg->mu,
                cfg->force ? cfg->force + b * blk : NULL, (double *)(soft + b * blk));
      }
    }
    free(wr);
    free(xq);
  }

  if (o->ddz) {
    for (int64_t k = 0; k < nsym; k++) {
      if (kk) { o->ddz[2 * k] = creal(soft[k]); o->ddz[2 * k + 1] = cimag(soft[k]); }
      else o->ddz[k] = creal(soft[k]);
    }
  }

  /* --- KK: per-block Viterbi-Viterbi phase over blocks b-1..b+1, unwrapped
   *     in multiples of pi/2, then derotation (unless the DD-LMS taps carry
   *     the phase) --- */
  if (kk && !cfg->dd_phase) {
    int64_t nb = nsym / blk;
    cplx *s4 = (cplx *)malloc(sizeof(cplx) * (size_t)nb);
    double *th = (double *)malloc(sizeof(double) * (size_t)nb);
    for (int64_t b = 0; b < nb; b++) {
      cplx a = 0.0;
      for (int64_t k = b * blk; k < (b + 1) * blk; k++) { cplx z2 = soft[k] * soft[k]; a += z2 * z2; }
      s4[b] = a;
    }
    rxo_vv_phase((double *)s4, nb, th);
    for (int64_t b = 0; b < nb; b++) {
      if (o->phase) o->phase[b] = th[b];
      cplx rv = cexp(-I * th[b]);
      for (int64_t k = b * blk; k < (b + 1) * blk; k++) soft[k] *= rv;
    }
    free(s4);
    free(th);
  }

  /* --- decisions, demapping, packing, error counting --- */
  const int64_t nbytes = (nsym * bps + 7) / 8;
  uint8_t *bits = (uint8_t *)calloc((size_t)nbytes, 1);
  int64_t cs = 0, se = 0, cb = 0, be = 0;
  for (int64_t k = 0; k < nsym; k++) {
    uint32_t b = symbol_bits(fmt, soft[k]);
    for (int j = 0; j < bps; j++) {
      int64_t t = k * bps + j;
      if ((b >> (bps - 1 - j)) & 1u) bits[t >> 3] |= (uint8_t)(1u << (t & 7));
    }
    if (k >= P + G && k < (cfg->count_end > 0 ? cfg->count_end : nsym - G)) {
      uint32_t r = (uint32_t)(rxo_splitmix64(cfg->seed, (uint64_t)k) >> (64 - bps));
      uint32_t d = r ^ b;
      int nerr = 0;
      for (; d; d &= d - 1) nerr++;
      cs++; cb += bps; be += nerr; se += nerr > 0;
    }
  }
  if (o->bits) memcpy(o->bits, bits, (size_t)nbytes);
  if (o->soft) {
    for (int64_t k = 0; k < nsym; k++) {
      if (kk) { o->soft[2 * k] = creal(soft[k]); o->soft[2 * k + 1] = cimag(soft[k]); }
      else o->soft[k] = creal(soft[k]);
    }
  }
  o->nbits = nsym * bps;
  o->counted_syms = cs; o->sym_errors = se; o->counted_bits = cb; o->bit_errors = be;
  free(bits); free(soft); free(w); free(ref); free(x); free(hm); free(code);
  return 0;
}

/*
 * Drives the FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_oracle_sanitize.py with gcc, host code only).
 *
 * Every optional output array is allocated at exactly the size rxo.h
 * documents, so a write past a documented size is an ASan report.  The run
 * covers one buffer through the full chain, the stream-continuation form
 * (the acquisition frozen from the first pass, a shortened counting window,
 * forced decisions), the frequency-domain front ends and the exported
 * building blocks with odd sizes.
 *
 * Input file: int32 fmt, rounding, form, equalizer; int64 n; uint64 seed;
 * then, when equalizer == 1, RXO_MLP_PARAMS doubles; then n*3/2 packed bytes.
 * Output file: the packed bits and error counts of both passes, as written
 * below (int64 nbits, sym_errors, bit_errors, then the bits).
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/rxo.h"

static void *take(size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
  memset(p, 0, bytes ? bytes : 1);
  return p;
}

static void read_all(FILE *f, void *dst, size_t bytes) {
  if (fread(dst, 1, bytes, f) != bytes) { fprintf(stderr, "short input\n"); exit(2); }
}

static void write_pass(FILE *f, const rxo_out *o, size_t nbytes) {
  const int64_t head[3] = {o->nbits, o->sym_errors, o->bit_errors};
  fwrite(head, sizeof head, 1, f);
  fwrite(o->bits, 1, nbytes, f);
}

int main(int argc, char **argv) {
  if (argc != 3) { fprintf(stderr, "usage: %s input output\n", argv[0]); return 2; }
  FILE *in = fopen(argv[1], "rb");
  if (!in) { perror(argv[1]); return 2; }
  int32_t hdr[4];
  int64_t n;
  uint64_t seed;
  read_all(in, hdr, sizeof hdr);
  read_all(in, &n, sizeof n);
  read_all(in, &seed, sizeof seed);
  double *mlp = NULL;
  if (hdr[3] == 1) {
    mlp = take(sizeof(double) * RXO_MLP_PARAMS);
    read_all(in, mlp, sizeof(double) * RXO_MLP_PARAMS);
  }
  uint8_t *packed = take((size_t)n * 3 / 2);
  read_all(in, packed, (size_t)n * 3 / 2);
  fclose(in);

  const int fmt = hdr[0], kk = fmt >= RXO_KK_QPSK;
  const int bps = fmt == RXO_PAM2 ? 1 : fmt == RXO_PAM8 ? 3 : fmt == RXO_KK_16QAM ? 4 : 2;
  const int64_t nsym = n / (kk ? 4 : 2);
  rxo_cfg cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.fmt = fmt;
  cfg.mf_taps = kk ? 65 : 33;
  cfg.ffe_taps = kk ? 21 : 15;
  cfg.prefix = 4096;
  cfg.hilbert_taps = 4097;
  cfg.os_log2 = 14;
  cfg.form = hdr[2];
  cfg.rounding = hdr[1];
  cfg.equalizer = hdr[3];
  cfg.rolloff = 0.1;
  cfg.mu = 1e-3;
  cfg.mu_cma = 1e-3;
  cfg.fc_over_fs = kk ? 0.55e9 / 4e9 : 0.0;
  cfg.seed = seed;
  cfg.mlp = mlp;

  /* every optional output, at its documented size */
  const size_t nbytes = (size_t)(nsym * bps + 7) / 8;
  rxo_out o;
  memset(&o, 0, sizeof o);
  if (kk) {
    o.field = take(sizeof(double) * 2 * (size_t)n);
    o.shifted = take(sizeof(double) * 2 * (size_t)n);
    o.mf = take(sizeof(double) * 2 * (size_t)(n / 2));
    o.soft = take(sizeof(double) * 2 * (size_t)nsym);
    o.ddz = take(sizeof(double) * 2 * (size_t)nsym);
    o.phase = take(sizeof(double) * (size_t)(nsym / 128));
  } else {
    o.mf = take(sizeof(double) * (size_t)n);
    o.timing = take(sizeof(double) * (size_t)(n / 512));
    o.xr = take(sizeof(double) * (size_t)n);
    o.soft = take(sizeof(double) * (size_t)nsym);
    o.ddz = take(sizeof(double) * (size_t)nsym);
  }
  o.taps = take(sizeof(double) * 2 * (size_t)cfg.ffe_taps);
  o.bits = take(nbytes);
  if (rxo_process(&cfg, packed, n, &o) != 0) { fprintf(stderr, "rejected\n"); return 3; }

  /* the stream form: acquisition frozen from the first pass, counting cut
   * short, every 97th decision forced to the lowest level */
  int32_t *force = take(sizeof(int32_t) * (size_t)nsym);
  for (int64_t k = 0; k < nsym; k++) force[k] = k % 97 == 50 && k > 4096 ? 0 : -1;
  rxo_out o2;
  memset(&o2, 0, sizeof o2);
  o2.bits = take(nbytes);
  o2.soft = take(sizeof(double) * (kk ? 2 : 1) * (size_t)nsym);
  cfg.frozen = &o;
  cfg.force = force;
  cfg.count_end = nsym - 1000;
  if (rxo_process(&cfg, packed, n, &o2) != 0) { fprintf(stderr, "rejected (stream form)\n"); return 3; }

  /* the frequency-domain front end (plain arithmetic, LMS only) */
  if (cfg.rounding == 0 && cfg.equalizer == 0) {
    rxo_out o3;
    memset(&o3, 0, sizeof o3);
    o3.bits = take(nbytes);
    o3.mf = take(sizeof(double) * (kk ? 2 * (size_t)(n / 2) : (size_t)n));
    if (!kk) {
      o3.xr = take(sizeof(double) * (size_t)n);
      o3.timing = take(sizeof(double) * (size_t)(n / 512));
    }
    cfg.front = 1;
    cfg.frozen = NULL;
    cfg.force = NULL;
    cfg.count_end = 0;
    if (kk) {   /* with the paper's 4-tap DD-LMS carrying the phase */
      cfg.ffe_taps = 4;
      cfg.dd_phase = 1;
    }
    if (rxo_process(&cfg, packed, n, &o3) != 0) { fprintf(stderr, "rejected (FD front end)\n"); return 3; }
    free(o3.bits); free(o3.mf); free(o3.xr); free(o3.timing);
  }

  /* building blocks at odd sizes */
  {
    double h[7], t[2 * 37], y[2 * 37];
    rxo_rrc_taps(7, 2.0, 0.5, h);
    for (int i = 0; i < 2 * 37; i++) t[i] = (double)((i * 7919) % 31) - 15.0;
    rxo_fir_same(t, 37, h, 7, y);
    rxo_fir_same_dec2_cplx(t, 36, h, 7, y);
    double f[2 * 8];
    for (int i = 0; i < 16; i++) f[i] = t[i];
    rxo_fft(f, 8, 0);
    rxo_fft(f, 8, 1);
    double hh[65], l[1000], phi[1000];
    rxo_hilbert_taps(65, hh);
    for (int i = 0; i < 1000; i++) l[i] = 0.001 * (double)((i * 37) % 101);
    rxo_hilbert_direct(l, 1000, hh, 65, phi);
    rxo_hilbert_os(l, 1000, hh, 65, 8, phi);
    rxo_hilbert_fd(l, 1000, phi);
    double yc[2 * 1000], xc[1000];
    for (int i = 0; i < 2000; i++) yc[i] = 0.01 * (double)((i * 17) % 23);
    rxo_fd_eq_dec2(yc, 1000, hh, 65, xc);
    double dd[2] = {0.3, -1.2}, xd[1000];
    rxo_fd_fir(l, 1000, hh, 65, xd);
    rxo_fd_delay(l, 1000, dd, xd);
    double x[1536], d[3], xr[1536], c[6];
    for (int i = 0; i < 1536; i++) x[i] = (double)((i * 13) % 7) - 3.0;
    rxo_gardner_sums(x, 1536, c);
    rxo_gardner(x, 1536, d);
    rxo_farrow(x, 1536, d, xr);
    double s4[2 * 5] = {1, 0, 0, 1, -1, 0, 0, -1, 1, 1}, ph[5];
    rxo_vv_phase(s4, 5, ph);
    double w[2 * 3] = {0}, ref[2 * 40], z[2 * 40];
    for (int i = 0; i < 80; i++) ref[i] = i % 2 ? 1.0 : -1.0;
    w[2] = 1.0;
    rxo_lms(t, 37, w, 3, 0, 16, ref, 2, 1, 1e-2, NULL, z);
    rxo_cma(t, 37, w, 3, 16, 1e-3, 2.0, 4, s4, z);
  }

  FILE *out = fopen(argv[2], "wb");
  if (!out) { perror(argv[2]); return 2; }
  write_pass(out, &o, nbytes);
  write_pass(out, &o2, nbytes);
  fclose(out);

  free(force); free(o2.bits); free(o2.soft);
  free(o.field); free(o.shifted); free(o.mf); free(o.soft); free(o.ddz); free(o.phase);
  free(o.timing); free(o.xr); free(o.taps); free(o.bits);
  free(packed); free(mlp);
  return 0;
}

// PAM front end for gfx950 (Sec. 2, first paragraph): DC removal, matched
// filter, blockwise clock-phase estimation, unwrapping and clock recovery.
#include "rx_dev.hpp"

#define PAM_TS 4096      // matched-filter outputs per tile (8 timing blocks)
#define PAM_MF_SUB 1     // tiles per workgroup (more serialises the tiles and loses parallel slack)
#define PAM_SUMW 16384   // samples per code-sum workgroup

// Exact integer sum of the codes (the buffer mean is then exact in FP64).
__global__ __launch_bounds__(256) void pam_sum(RxLaunch L) {
  __shared__ uint32_t red[4];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int64_t base = (int64_t)blockIdx.x * PAM_SUMW;
  if (base >= n) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) J.sc->t_start = (unsigned long long)wall_clock64();   // buffer start
  uint32_t s = 0;
  for (int g = threadIdx.x; g < PAM_SUMW / 8; g += 256) {
    const int64_t s0 = base + 8 * g;
    if (s0 + 8 <= n) {
      int c[8];
      read_codes8(L.in[jb], s0 >> 3, c);
#pragma unroll
      for (int e = 0; e < 8; e++) s += (uint32_t)c[e];
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) J.upart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// The buffer mean of v = code + 0.5 from the code-sum partials, once per
// buffer (exact integer sum, FP64 division).
__global__ __launch_bounds__(256) void pam_mean(RxLaunch L) {
  __shared__ unsigned long long rs[4];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int64_t np = (n + PAM_SUMW - 1) / PAM_SUMW;
  unsigned long long s = 0;
  for (int64_t i = threadIdx.x; i < np; i += 256) s += J.upart[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) rs[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    J.sc->mean_re = (double)(rs[0] + rs[1] + rs[2] + rs[3]) / (double)n + 0.5;
    J.sc->mean_im = 0.0;
  }
}

__device__ __forceinline__ int xpad(int i) { return i + (i >> 4); }

// x0 = v - mean(v); y = MF(x0) (33 taps, centred, zero outside); partial
// sums of y^2; Gardner detector sums per 512-sample block on y (the AGC gain
// does not change the angle of the sums).
__global__ __launch_bounds__(256) void pam_mf(RxLaunch L) {
  constexpr int XN = PAM_TS + 40;   // x0 over [t0-20, t0+TS+20)
  constexpr int YN = PAM_TS + 8;    // y over [t0-4, t0+TS+4)
  __shared__ float xs[XN + XN / 16 + 1];
  __shared__ float ys[YN];
  __shared__ double red[4];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const uint8_t *in = L.in[jb];
  if ((int64_t)blockIdx.x * PAM_MF_SUB * PAM_TS >= n) return;
  // a stream buffer after the first starts here (its DC mean is the stream's)
  if (L.s0[jb] >= 0 && blockIdx.x == 0 && threadIdx.x == 0) J.sc->t_start = (unsigned long long)wall_clock64();
  float hmf[33];   // the taps, read at the start (uniform: scalar registers)
#pragma unroll
  for (int i = 0; i < 33; i++) hmf[i] = J.mf[i];
  const double mv = J.sc->mean_re;   // from pam_mean
  const float mvh = (float)(mv - 0.5);
  constexpr int NGR = (PAM_TS + 48) / 8, GPT = (NGR + 255) / 256;   // code groups per tile and thread
  const int64_t gmax = n / 8 - 1;
  for (int sub = 0; sub < PAM_MF_SUB; sub++) {
    const int64_t tile = (int64_t)blockIdx.x * PAM_MF_SUB + sub;
    const int64_t t0 = tile * PAM_TS;
    if (t0 >= n) break;
    __syncthreads();   // the previous tile's readers of xs and ys are done
    // codes of [t0 - 24, t0 + TS + 24) in aligned groups of eight (t0 is a
    // multiple of 8); xs[i] holds sample t0 - 20 + i.  Every group read is
    // issued first (group index clamped into the buffer); groups past a
    // buffer edge are re-read sample by sample.
    uint32_t raw[GPT][3];
#pragma unroll
    for (int gi = 0; gi < GPT; gi++) {
      const int g = threadIdx.x + 256 * gi;
      if (g < NGR) {
        const int64_t gg = (t0 - 24) / 8 + g;
        const uint32_t *p = reinterpret_cast<const uint32_t *>(in + 12 * (gg < 0 ? 0 : (gg > gmax ? gmax : gg)));
        raw[gi][0] = p[0];
        raw[gi][1] = p[1];
        raw[gi][2] = p[2];
      }
    }
#pragma unroll
    for (int gi = 0; gi < GPT; gi++) {
      const int g = threadIdx.x + 256 * gi;
      if (g >= NGR) break;
      const int64_t s0 = t0 - 24 + 8 * g;
      int c[8];
      if (s0 >= 0 && s0 + 8 <= n) {
        unpack_codes8(raw[gi][0], raw[gi][1], raw[gi][2], c);
      } else {
#pragma unroll
        for (int e = 0; e < 8; e++) c[e] = (s0 + e >= 0 && s0 + e < n) ? read_code(in, s0 + e) : -1;
      }
      // x0 = c + 0.5 - mean = c - (mean - 1/2), the latter rounded to FP32 once
      float xv[8];
#pragma unroll
      for (int e = 0; e < 8; e++) xv[e] = c[e] >= 0 ? (float)c[e] - mvh : 0.0f;
      // xs index i = ib + e, ib = 8 g - 4; xpad(i) = i + i / 16, and the run
      // of eight crosses a pad (after e = 3) exactly when g is even
      const int ib = 8 * g - 4;
      if (g >= 1 && ib + 8 <= XN) {
        float *const xp = xs + ib + (ib >> 4);
        const int cross = (g & 1) ^ 1;
#pragma unroll
        for (int e = 0; e < 8; e++) xp[e + (e >= 4 ? cross : 0)] = xv[e];
      } else {
#pragma unroll
        for (int e = 0; e < 8; e++)
          if (ib + e >= 0 && ib + e < XN) xs[xpad(ib + e)] = xv[e];
      }
    }
    __syncthreads();
    // 16 consecutive outputs per thread: y[t0 + 16 tid + o] from 48 inputs
    double p2 = 0.0;
    {
      float acc[16];
#pragma unroll
      for (int o = 0; o < 16; o++) acc[o] = 0.0f;
      // xpad(16 tid + 4 + d) = 17 tid + (4 + d) + (4 + d) / 16: a per-thread base and
      // immediate offsets
      const float *xb = xs + 17 * threadIdx.x;
#pragma unroll
      for (int d = 0; d < 48; d++) {
        const float v = xb[(4 + d) + ((4 + d) >> 4)];
#pragma unroll
        for (int o = 0; o < 16; o++) {
          const int tap = o + 32 - d;
          if (tap >= 0 && tap <= 32) acc[o] = fmaf(hmf[tap], v, acc[o]);
        }
      }
      float q2 = 0.0f;   // 16 squares in FP32, then one FP64 add
      const int64_t rem = n - (t0 + 16 * (int64_t)threadIdx.x);
      const int lim = rem < 0 ? 0 : (rem > 16 ? 16 : (int)rem);   // this thread's outputs inside the buffer
#pragma unroll
      for (int o = 0; o < 16; o++) {
        const float yv = o < lim ? acc[o] : 0.0f;
        ys[16 * threadIdx.x + o + 4] = yv;
        q2 = fmaf(yv, yv, q2);
      }
      p2 = q2;
    }
    if (threadIdx.x < 8) {   // the 4 outputs either side of the tile
      const int l = threadIdx.x < 4 ? (int)threadIdx.x - 4 : PAM_TS + (int)threadIdx.x - 4;
      const int64_t t = t0 + l;
      float a = 0.0f;
#pragma unroll
      for (int i = 0; i < 33; i++) a = fmaf(hmf[i], xs[xpad(l + 36 - i)], a);
      ys[l + 4] = (t >= 0 && t < n) ? a : 0.0f;
    }
    p2 = block_sum(p2, red);   // (its barriers also publish ys)
    if (threadIdx.x == 0) J.part2[tile] = p2;
    {   // coalesced copy-out of the tile (32-bit offsets from its start)
      const auto yo = gptr(J.y) + t0;
      const int cnt = (int)(n - t0 < PAM_TS ? n - t0 : PAM_TS);
      for (int i = threadIdx.x; i < cnt; i += 256) yo[i] = ys[i + 4];
    }
    // Gardner sums: 8 blocks of 256 symbols, 32 threads x 8 symbols each.
    const int bl = threadIdx.x >> 5, gsub = threadIdx.x & 31;
    float g0 = 0.0f, g1 = 0.0f;
    for (int e = 0; e < 8; e++) {
      const int s = 2 * (256 * bl + 8 * gsub + e) + 4;   // ys index of the symbol sample
      const float y0 = ys[s], y1 = ys[s + 1], y2 = ys[s + 2];
      g0 += y1 * (y0 - y2);
      const float ym = ys[s - 1], y3 = ys[s + 3], y4 = ys[s + 4];
      const float h0 = (-ym + 9.0f * y0 + 9.0f * y1 - y2) * 0.0625f;
      const float h1 = (-y0 + 9.0f * y1 + 9.0f * y2 - y3) * 0.0625f;
      const float h2 = (-y1 + 9.0f * y2 + 9.0f * y3 - y4) * 0.0625f;
      g1 += h1 * (h0 - h2);
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      g0 += __shfl_xor(g0, o, 32);
      g1 += __shfl_xor(g1, o, 32);
    }
    const int64_t gb = t0 / 512 + bl;
    if (gsub == 0 && gb * 512 < n) J.gard[gb] = make_float2(g0, g1);
  }
}

// Angle of the detector sums averaged over blocks b-16 .. b+16.  The
// quarter-symbol detector's samples come from the half-sample cubic
// interpolator, whose gain at half the symbol rate is 5 / (4 sqrt 2); its
// sums are scaled by the inverse squared gain, 32/25, so that both
// detectors weigh the same in the angle.
__global__ __launch_bounds__(256) void pam_gavg(RxLaunch L) {
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t nb = L.n[jb] / 512;
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= nb) return;
  double re = 0.0, im = 0.0;
  const int64_t lo = b - 16 < 0 ? 0 : b - 16, hi = b + 16 >= nb ? nb - 1 : b + 16;
  for (int64_t j = lo; j <= hi; j++) {
    re += J.gard[j].x;
    im += J.gard[j].y;
  }
  J.delta[nb + b] = (float)atan2(im * (32.0 / 25.0), re);   // raw angle, second half of the array
}

// Unwrap (wrapped differences + workgroup prefix sum), timing shift
// delta_b = 1/2 + psi_b / pi samples, and the AGC gain.  A stream buffer
// after the first keeps the stream's gain and continues the unwrap from the
// angle carried from the previous buffer's last emitted timing block (the
// block just before its first emitted sample: the clock-phase continuity of
// the paper's stream-to-stream events); every stream buffer carries its own
// last emitted block's angle on.
__global__ __launch_bounds__(1024) void pam_unwrap(RxLaunch L) {
  __shared__ double scan[1024];
  __shared__ double red[16];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int nb = (int)(n / 512);
  const float *raw = J.delta + nb;
  const bool cont = J.stream && L.s0[jb] >= 0;
  if (!cont) {
    // power partials: one per matched-filter tile, or per pair of
    // 512-sample blocks from the frequency-domain equaliser
    const int64_t pt = J.fft_log2 == RX_KK_FD_LOG2 ? 1024 : PAM_TS;
    const int64_t np = (n + pt - 1) / pt;
    double p = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += 1024) p += J.part2[i];
    p = block_sum(p, red);
    if (threadIdx.x == 0) J.sc->agc = 1.0 / sqrt(p / (double)n);
  }
  const RxSpan sp = rx_span(J, n, L.s0[jb]);
  const int bs = cont ? (int)(2 * sp.k_lo / 512) - 1 : 0;   // first block of the unwrap
  const int blast = (int)(2 * sp.k_hi / 512) - 1;           // last emitted timing block
  const double first = cont ? J.sc->acc_carry : 0.0;
  const int per = (nb + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  constexpr double TWO_PI = 6.283185307179586;
  auto wrap = [&](double d) { return d - TWO_PI * floor(d / TWO_PI + 0.5); };
  auto step = [&](int b) -> double {
    if (b < bs) return 0.0;
    if (b == bs) return cont ? first : (double)raw[b];
    return wrap((double)raw[b] - raw[b - 1]);
  };
  double local = 0.0;
  for (int b = b0; b < b0 + per && b < nb; b++) local += step(b);
  scan[threadIdx.x] = local;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const double v = threadIdx.x >= o ? scan[threadIdx.x - o] : 0.0;
    __syncthreads();
    scan[threadIdx.x] += v;
    __syncthreads();
  }
  double acc = scan[threadIdx.x] - local;   // exclusive prefix
  // raw angles live in the second half of the array, shifts in the first
  for (int b = b0; b < b0 + per && b < nb; b++) {
    acc += step(b);
    J.delta[b] = (float)(0.5 + acc / 3.141592653589793);
    if (J.stream && b == blast) J.sc->acc_carry = acc;
  }
}

// Cubic-Lagrange (Farrow) interpolation with the AGC gain:
// xr[t] = g * y(t + delta_b), t in block b.  A workgroup covers FAR_SPAN
// consecutive samples (FAR_SPAN / 512 timing blocks), one sample per thread
// and pass; the four Lagrange weights are formed once per block (each pair of
// passes stays in one block), offsets are 32-bit from the span's start.
#define FAR_SPAN 8192
__global__ __launch_bounds__(256) void pam_farrow(RxLaunch L) {
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int64_t base = (int64_t)blockIdx.x * FAR_SPAN;
  if (base >= n) return;
  const float g = (float)J.sc->agc;
  const auto y = gptr(J.y) + base;
  const auto xr = gptr(J.xr) + base;
  const auto dl = gptr(J.delta) + base / 512;
  const int span = (int)(n - base < FAR_SPAN ? n - base : FAR_SPAN);   // multiple of 1024
  const int lo = (int)(base < 4 ? -base : -4), hi = (int)(n - base < FAR_SPAN + 4 ? n - base : FAR_SPAN + 4);
  constexpr int NB = FAR_SPAN / 512;   // timing blocks per span
  const int nblk = span / 512;
  float dv[NB];   // every block's offset first (uniform values)
#pragma unroll
  for (int k = 0; k < NB; k++) dv[k] = k < nblk ? dl[k] : 0.0f;
  // block o2: its four taps i0 - 1 .. i0 + 2 of both passes, when the whole
  // block's taps lie inside the buffer (relative to base: [lo, hi)); the
  // next block's reads are issued before the current block is finished
  auto fetch = [&](int o2, float (&yv)[2][4]) {
    const int sh = (int)floorf(dv[o2]);
    const bool inside = 512 * o2 + sh - 1 >= lo && 512 * o2 + 511 + sh + 2 < hi;
    if (inside) {
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const int i0 = 512 * o2 + 256 * h + threadIdx.x + sh;
#pragma unroll
        for (int k = 0; k < 4; k++) yv[h][k] = y[i0 - 1 + k];
      }
    }
    return inside;
  };
  float ya[2][4], yb[2][4];
  bool ina = fetch(0, ya);
#pragma unroll
  for (int o2 = 0; o2 < NB; o2++) {   // block o2 of the span: passes 2 o2, 2 o2 + 1
    if (o2 >= nblk) break;
    bool inb = false;
    if (o2 + 1 < nblk) inb = fetch(o2 + 1, yb);
    const float d = dv[o2];
    const float fl = floorf(d), mu = d - fl;
    const int sh = (int)fl;
    const float lm1 = -mu * (mu - 1.0f) * (mu - 2.0f) * (1.0f / 6.0f);
    const float l0 = (mu + 1.0f) * (mu - 1.0f) * (mu - 2.0f) * 0.5f;
    const float l1 = -(mu + 1.0f) * mu * (mu - 2.0f) * 0.5f;
    const float l2 = (mu + 1.0f) * mu * (mu - 1.0f) * (1.0f / 6.0f);
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int t = 512 * o2 + 256 * h + threadIdx.x;
      const int i0 = t + sh;
      float v;
      if (ina) {
        v = lm1 * ya[h][0] + l0 * ya[h][1] + l1 * ya[h][2] + l2 * ya[h][3];
      } else {
        auto yat = [&](int j) { return (base + j >= 0 && base + j < n) ? y[j] : 0.0f; };
        v = lm1 * yat(i0 - 1) + l0 * yat(i0) + l1 * yat(i0 + 1) + l2 * yat(i0 + 2);
      }
      xr[t] = g * v;
    }
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
      for (int k = 0; k < 4; k++) ya[h][k] = yb[h][k];
    ina = inb;
  }
}

void rx_launch_pam_stage(int stage, const RxLaunch &L, int64_t maxn, int log2n, hipStream_t s) {
  const unsigned cnt = (unsigned)L.count;
  if (log2n == RX_KK_FD_LOG2 && (stage == ST_PAM_MF || stage == ST_PAM_FARROW)) {
    rx_launch_pamfd(stage, L, maxn, s);
    return;
  }
  const int64_t nb = maxn / 512;
  switch (stage) {
    case ST_PAM_SUM:
      hipLaunchKernelGGL(pam_sum, dim3((unsigned)((maxn + PAM_SUMW - 1) / PAM_SUMW), cnt), dim3(256), 0, s, L);
      hipLaunchKernelGGL(pam_mean, dim3(1, cnt), dim3(256), 0, s, L);
      break;
    case ST_PAM_MF:
      hipLaunchKernelGGL(pam_mf, dim3((unsigned)((maxn + PAM_MF_SUB * PAM_TS - 1) / (PAM_MF_SUB * PAM_TS)), cnt),
                         dim3(256), 0, s, L);
      break;
    case ST_PAM_GAVG:
      hipLaunchKernelGGL(pam_gavg, dim3((unsigned)((nb + 255) / 256), cnt), dim3(256), 0, s, L);
      break;
    case ST_PAM_UNWRAP:
      hipLaunchKernelGGL(pam_unwrap, dim3(1, cnt), dim3(1024), 0, s, L);
      break;
    case ST_PAM_FARROW:
      hipLaunchKernelGGL(pam_farrow, dim3((unsigned)((maxn + FAR_SPAN - 1) / FAR_SPAN), cnt), dim3(256), 0, s, L);
      break;
  }
}

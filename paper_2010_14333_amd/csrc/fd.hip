// Kramers-Kronig front end in the paper's own frequency-domain form
// (Sec. 2, second paragraph: Hilbert transform with a 1024-point FFT and
// IFFT, field and downshift, a static equaliser on a 1024-point FFT, a
// 512-point IFFT to 2 samples per symbol; first paragraph: 1024-point
// transforms with "100 % overlap", 8192 blocks per 2^22-sample buffer).
//
// Block b covers samples 512 b - 256 .. 512 b + 767 and contributes its 512
// central samples (and their 256 outputs at 2 samples per symbol).  A
// 1024-point transform is one wavefront's work: 16 points per lane, the
// passes exchanging through the wavefront's own LDS, so each workgroup is a
// single wavefront and its barriers cost nothing.
//
//  kkfd_hilbert  two real blocks of l = ln sqrt(v) per complex transform
//                (block A in the real part, B in the imaginary part),
//                times -j sgn(k), back: the phase of every central sample
//                (written, in revolutions) and per-pair sums of the field E
//  kkfd_mean     the carrier mean m = sum E / n, per buffer (FP64)
//  kkfd_eq       per block: E from the codes and phases, y = (E - m) D with
//                the downshift phase frac(r t) in FP64, its 1024-point
//                spectrum times the equaliser's response, the 512 bins of
//                |f| < fs/4 through a 512-point transform (three radix-8
//                passes), the central 256 outputs
//
// The output is carrier-free; the consumers' carrier term vanishes (the job
// carries a zero carrier response).  The per-block sums keep the layout the
// prefix stage reads: (sum E), (sum |Z|^2, 0), (0, 0).
#include "fft_lds.hpp"

namespace {
constexpr int FN = 1024, FHOP = 512, FGUARD = 256, FT = 64;

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Last pass of the Hilbert transform's forward FFT: Y = Z H with H = -j S,
// S[k] = sgn(k) / N, taken into registers as conj(Y) (the inverse runs as a
// forward transform of the conjugate): output k = threadIdx.x + i T to y[i].
struct SpecOut {
  const float *s;
  float2 (&y)[16];
  float hs[16];
  __device__ __forceinline__ void begin() {
#pragma unroll
    for (int i = 0; i < 16; i++) hs[i] = gptr(s)[threadIdx.x + i * FT];
  }
  __device__ __forceinline__ void operator()(int koff, int, float2 z) const {
    const int i = koff / FT;
    y[i] = make_float2(z.y * hs[i], z.x * hs[i]);
  }
};

// Last pass of the inverse: output k = threadIdx.x + i T is phiA - j phiB of
// block sample k, kept in revolutions (sgn / (2 pi) applied).
struct PhaseOut {
  float (&pa)[16];
  float (&pb)[16];
  float sgnrev;
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ void operator()(int koff, int, float2 v) const {
    const int i = koff / FT;
    pa[i] = v.x * sgnrev;
    pb[i] = -v.y * sgnrev;
  }
};

// Last pass of the equaliser's forward FFT: bin k times the response (real:
// the taps are symmetric; 1 / N folded in), kept when k < N/4 or k >= 3N/4,
// conjugated into the 512-point transform's input at k' = k or k - N/2 in
// the same LDS buffer: the workgroup is one wavefront, whose lanes have all
// read their last-pass inputs before any of them writes.
struct EqOut {
  const float *hq;
  float2 *dst;
  float w[16];
  __device__ __forceinline__ void begin() {
#pragma unroll
    for (int i = 0; i < 16; i++) w[i] = gptr(hq)[threadIdx.x + i * FT];
  }
  __device__ __forceinline__ void operator()(int koff, int, float2 v) const {
    const int k = (int)threadIdx.x + koff, i = koff / FT;
    if (k < FN / 4) dst[fpad(k)] = make_float2(v.x * w[i], -v.y * w[i]);
    else if (k >= 3 * FN / 4) dst[fpad(k - FN / 2)] = make_float2(v.x * w[i], -v.y * w[i]);
  }
};

// Last pass of the 512-point transform: output m' = threadIdx.x + r T is the
// conjugate of the filtered block's sample 2 m'; the central ones are kept.
struct DecOut {
  float2 (&z)[8];
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ void operator()(int koff, int, float2 v) const { z[koff / FT] = make_float2(v.x, -v.y); }
};
}   // namespace

__global__ __launch_bounds__(FT) void kkfd_hilbert(RxLaunch L) {
  __shared__ float2 lds[FN + FN / 16];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int64_t b0 = 2 * (int64_t)blockIdx.x;
  if (b0 * FHOP >= n) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) J.sc->t_start = (unsigned long long)wall_clock64();   // buffer start
  const uint8_t *in = L.in[jb];
  const int64_t F[2] = {b0 * FHOP - FGUARD, (b0 + 1) * FHOP - FGUARD};
  const int j = threadIdx.x;
  // the codes of samples F + j + 64 r: the inputs of this lane's first
  // butterfly, and (the same samples) the ones whose phases it receives
  int ca[16], cb[16];
#pragma unroll
  for (int r = 0; r < 16; r++) {
    ca[r] = read_code(in, clampi(F[0] + j + FT * r, 0, n - 1));
    cb[r] = read_code(in, clampi(F[1] + j + FT * r, 0, n - 1));
  }
  // l - l_ref, l = ln sqrt(v) = (ln 2 / 2) log2(v) (the transform is zero at
  // DC, so the block's own reference sample leaves the phase unchanged)
  constexpr float HLN2 = 0.34657359027997264f;
  const float lr0 = __builtin_amdgcn_logf((float)read_code(in, clampi(F[0] + FN / 2, 0, n - 1)) + 0.5f);
  const float lr1 = __builtin_amdgcn_logf((float)read_code(in, clampi(F[1] + FN / 2, 0, n - 1)) + 0.5f);
  {
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; r++)
      v[r] = make_float2(HLN2 * (__builtin_amdgcn_logf((float)ca[r] + 0.5f) - lr0),
                         HLN2 * (__builtin_amdgcn_logf((float)cb[r] + 0.5f) - lr1));
    dft16(v);
    const int p0 = fpad(16 * j);
#pragma unroll
    for (int r = 0; r < 16; r++) lds[p0 + r] = v[r];
  }
  __syncthreads();
  {
    float2 y[16];
    fft_passes<FN, 16, false>(lds, J.twid, SpecOut{J.hspec, y, {}});
    dft16(y);   // the inverse's first pass: its inputs j + r T are this lane's outputs
    __syncthreads();
    const int p0 = fpad(16 * j);
#pragma unroll
    for (int r = 0; r < 16; r++) lds[p0 + r] = y[r];
  }
  __syncthreads();
  float pa[16], pb[16];
  const float sgnrev = J.sgn * 0.15915494309189535f;
  fft_passes<FN, 16, false>(lds, J.twid, PhaseOut{pa, pb, sgnrev});
  // central samples: block index k = j + 64 i, i = 4 .. 11
  float ser = 0.0f, sei = 0.0f;
#pragma unroll
  for (int x = 0; x < 2; x++) {
#pragma unroll
    for (int i = FGUARD / FT; i < (FGUARD + FHOP) / FT; i++) {
      const int64_t t = F[x] + j + FT * i;
      if (t < n) {
        const float ph = x ? pb[i] : pa[i];
        const int c = x ? cb[i] : ca[i];
        const float2 e = cscale(cis_rev(ph), __builtin_amdgcn_sqrtf((float)c + 0.5f));
        gptr(J.phi)[t] = ph;
        ser += e.x;
        sei += e.y;
        if (J.field) gstore(J.field, t, e);
      }
    }
  }
  const double sr = wave_sum((double)ser), si = wave_sum((double)sei);
  if (threadIdx.x == 0) J.fdpart[blockIdx.x] = make_double2(sr, si);
}

__global__ __launch_bounds__(256) void kkfd_mean(RxLaunch L) {
  __shared__ double red[2 * 4];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb], np = (n + 2 * FHOP - 1) / (2 * FHOP);
  double v[2] = {0.0, 0.0};
  for (int64_t i = threadIdx.x; i < np; i += 256) {
    v[0] += J.fdpart[i].x;
    v[1] += J.fdpart[i].y;
  }
  block_sum_n<2>(v, red);
  if (threadIdx.x == 0) {
    J.sc->mean_re = v[0] / (double)n;
    J.sc->mean_im = v[1] / (double)n;
  }
}

__global__ __launch_bounds__(FT) void kkfd_eq(RxLaunch L) {
  __shared__ float2 lds[FN + FN / 16];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int64_t b = blockIdx.x;
  if (b * FHOP >= n) return;
  const uint8_t *in = L.in[jb];
  const int j = threadIdx.x;
  const int64_t t0 = b * FHOP - FGUARD + j;   // this lane's samples t0 + 64 r
  const float2 mean = make_float2((float)J.sc->mean_re, (float)J.sc->mean_im);
  // the downshift phasor from an FP64 anchor, then one fixed rotation per
  // 64 samples (15 steps)
  float2 dph = cis_rev(-downshift_rev(J.r, t0));
  const float2 drot = cis_rev(-downshift_rev(J.r, FT));
  float ser = 0.0f, sei = 0.0f;
  {
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int64_t t = t0 + FT * r;
      v[r] = make_float2(0.0f, 0.0f);
      if (t >= 0 && t < n) {
        const int c = read_code(in, t);
        const float2 e = cscale(cis_rev(gptr(J.phi)[t]), __builtin_amdgcn_sqrtf((float)c + 0.5f));
        if (r >= FGUARD / FT && r < (FGUARD + FHOP) / FT) {
          ser += e.x;
          sei += e.y;
        }
        v[r] = cmul(csub(e, mean), dph);
      }
      dph = cmul(dph, drot);
    }
    dft16(v);
    const int p0 = fpad(16 * j);
#pragma unroll
    for (int r = 0; r < 16; r++) lds[p0 + r] = v[r];
  }
  __syncthreads();
  fft_passes<FN, 16, true>(lds, J.twid, EqOut{J.hspec + FN, lds, {}});
  float2 z[8];
  fft_passes8<FN / 2, 1, false>(lds, J.twid + FN, DecOut{z});
  // outputs m' = j + 64 r of the block; its central ones are r = 2 .. 5
  float zz = 0.0f;
#pragma unroll
  for (int r = FGUARD / 2 / FT; r < (FGUARD + FHOP) / 2 / FT; r++) {
    const int64_t m = b * (FHOP / 2) - FGUARD / 2 + j + FT * r;
    if (2 * m < n) {
      gstore(J.z, m, z[r]);
      zz = fmaf(z[r].x, z[r].x, fmaf(z[r].y, z[r].y, zz));
    }
  }
  const double s0 = wave_sum((double)ser), s1 = wave_sum((double)sei), s2 = wave_sum((double)zz);
  if (threadIdx.x == 0) {
    J.part[3 * b] = make_double2(s0, s1);
    J.part[3 * b + 1] = make_double2(s2, 0.0);
    J.part[3 * b + 2] = make_double2(0.0, 0.0);
  }
}

void rx_launch_kkfd(const RxLaunch &L, int64_t maxn, hipStream_t s) {
  const unsigned cnt = (unsigned)L.count;
  const int64_t nb = (maxn + FHOP - 1) / FHOP;
  hipLaunchKernelGGL(kkfd_hilbert, dim3((unsigned)((nb + 1) / 2), cnt), dim3(FT), 0, s, L);
  hipLaunchKernelGGL(kkfd_mean, dim3(1, cnt), dim3(256), 0, s, L);
  hipLaunchKernelGGL(kkfd_eq, dim3((unsigned)nb, cnt), dim3(FT), 0, s, L);
}

// ---- PAM (Sec. 2, first paragraph): the 503-tap static equaliser on the
// 1024-point blocks and the clock recovery in the frequency domain.  Two
// real blocks per complex transform again (A real, B imaginary).
namespace {
// Last pass of the forward transform: conj(Z H) with the real response H
// (1/N folded in) into registers, the inverse's input.
struct RealEqOut {
  const float *hq;
  float2 (&y)[16];
  float w[16];
  __device__ __forceinline__ void begin() {
#pragma unroll
    for (int i = 0; i < 16; i++) w[i] = gptr(hq)[threadIdx.x + i * FT];
  }
  __device__ __forceinline__ void operator()(int koff, int, float2 z) const {
    const int i = koff / FT;
    y[i] = make_float2(z.x * w[i], -z.y * w[i]);
  }
};
// Last pass of the inverse: block sample k = threadIdx.x + i T of A and B.
struct PairOut {
  float (&a)[16];
  float (&b)[16];
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ void operator()(int koff, int, float2 v) const {
    const int i = koff / FT;
    a[i] = v.x;
    b[i] = -v.y;
  }
};
}   // namespace

// y = the static equaliser's output at every central sample (written, before
// the AGC gain), the power partial of the pair, and each block's Gardner
// detector sums (the detector reads y up to 4 samples past the block, which
// the transform's outputs cover: a 503-tap output is exact up to 251 samples
// from the block's ends).
__global__ __launch_bounds__(FT) void pamfd_eq(RxLaunch L) {
  __shared__ float2 lds[FN + FN / 16];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int64_t b0 = 2 * (int64_t)blockIdx.x;
  if (b0 * FHOP >= n) return;
  const uint8_t *in = L.in[jb];
  const int64_t F[2] = {b0 * FHOP - FGUARD, (b0 + 1) * FHOP - FGUARD};
  const int j = threadIdx.x;
  const float off = (float)(J.sc->mean_re - 0.5);   // x0 = code - (mean - 1/2)
  {
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int64_t ta = F[0] + j + FT * r, tb = F[1] + j + FT * r;
      v[r] = make_float2(ta >= 0 && ta < n ? (float)read_code(in, ta) - off : 0.0f,
                         tb >= 0 && tb < n ? (float)read_code(in, tb) - off : 0.0f);
    }
    dft16(v);
    const int p0 = fpad(16 * j);
#pragma unroll
    for (int r = 0; r < 16; r++) lds[p0 + r] = v[r];
  }
  __syncthreads();
  {
    float2 y[16];
    fft_passes<FN, 16, false>(lds, J.twid, RealEqOut{J.hspec + FN, y, {}});
    dft16(y);
    __syncthreads();
    const int p0 = fpad(16 * j);
#pragma unroll
    for (int r = 0; r < 16; r++) lds[p0 + r] = y[r];
  }
  __syncthreads();
  float ya[16], yb[16];
  fft_passes<FN, 16, false>(lds, J.twid, PairOut{ya, yb});
  __syncthreads();
  // y of block samples 192 .. 831 of both blocks into LDS (zero outside the
  // buffer, as the detector takes it), the central ones to HBM
  float *ys = reinterpret_cast<float *>(lds);
  constexpr int YLO = 3 * FT, YN = 10 * FT;
  float p2 = 0.0f;
#pragma unroll
  for (int x = 0; x < 2; x++) {
#pragma unroll
    for (int i = 3; i < 13; i++) {
      const int64_t t = F[x] + j + FT * i;
      const float yv = (t >= 0 && t < n) ? (x ? yb[i] : ya[i]) : 0.0f;
      ys[x * YN + j + FT * i - YLO] = yv;
      if (i >= FGUARD / FT && i < (FGUARD + FHOP) / FT && t < n) {
        gptr(J.y)[t] = yv;
        p2 = fmaf(yv, yv, p2);
      }
    }
  }
  __syncthreads();
  // Gardner sums of each block: its 256 symbols, 4 per lane; symbol sample
  // s = 2 k sits at block sample 2 k - 512 b + 256
#pragma unroll
  for (int x = 0; x < 2; x++) {
    float g0 = 0.0f, g1 = 0.0f;
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int s = x * YN + FGUARD + 2 * (4 * j + e) - YLO;
      const float ym = ys[s - 1], y0 = ys[s], y1 = ys[s + 1], y2 = ys[s + 2], y3 = ys[s + 3], y4 = ys[s + 4];
      g0 += y1 * (y0 - y2);
      const float h0 = (-ym + 9.0f * y0 + 9.0f * y1 - y2) * 0.0625f;
      const float h1 = (-y0 + 9.0f * y1 + 9.0f * y2 - y3) * 0.0625f;
      const float h2 = (-y1 + 9.0f * y2 + 9.0f * y3 - y4) * 0.0625f;
      g1 += h1 * (h0 - h2);
    }
    g0 = wave_sum(g0);
    g1 = wave_sum(g1);
    if (threadIdx.x == 0 && (b0 + x) * FHOP < n) J.gard[b0 + x] = make_float2(g0, g1);
  }
  const float ps = wave_sum(p2);
  if (threadIdx.x == 0) J.part2[blockIdx.x] = (double)ps;
}

// xr = g y(t + delta_b) for the central samples of block b: the pair's
// spectrum Z = A + j B is split into the two blocks' spectra, A[k] =
// (Z[k] + conj Z[N-k]) / 2 and B[k] = (Z[k] - conj Z[N-k]) / 2j, each takes
// its own block's delay exp(+j 2 pi k delta / N) (signed k; cos(pi delta)
// at N/2, so both stay real), and A' + j B' goes back.
__global__ __launch_bounds__(FT) void pamfd_clock(RxLaunch L) {
  __shared__ float2 lds[FN + FN / 16];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int64_t b0 = 2 * (int64_t)blockIdx.x;
  if (b0 * FHOP >= n) return;
  const int64_t F[2] = {b0 * FHOP - FGUARD, (b0 + 1) * FHOP - FGUARD};
  const int j = threadIdx.x;
  const auto yin = gptr(J.y);
  {
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int64_t ta = F[0] + j + FT * r, tb = F[1] + j + FT * r;
      v[r] = make_float2(ta >= 0 && ta < n ? yin[ta] : 0.0f, tb >= 0 && tb < n ? yin[tb] : 0.0f);
    }
    dft16(v);
    const int p0 = fpad(16 * j);
#pragma unroll
    for (int r = 0; r < 16; r++) lds[p0 + r] = v[r];
  }
  __syncthreads();
  fft_passes<FN, 16, true>(lds, J.twid, LdsOut{lds});   // Z in natural order
  const float da = J.delta[b0], db = (b0 + 1) * FHOP < n ? J.delta[b0 + 1] : 0.0f;
  const float g = (float)J.sc->agc * (1.0f / FN);
  float2 w[16];
#pragma unroll
  for (int i = 0; i < 16; i++) {
    const int k = j + FT * i;
    const float2 zk = lds[fpad(k)], zm = lds[fpad((FN - k) & (FN - 1))];
    const float2 a = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));   // A[k]
    const float2 bb = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));  // B[k]
    float2 ra, rb;
    if (k == FN / 2) {
      ra = make_float2(__builtin_amdgcn_cosf(0.5f * da), 0.0f);
      rb = make_float2(__builtin_amdgcn_cosf(0.5f * db), 0.0f);
    } else {
      const float ks = (float)(k < FN / 2 ? k : k - FN) * (1.0f / FN);
      ra = cis_rev(ks * da);
      rb = cis_rev(ks * db);
    }
    const float2 pa = cmul(a, ra), pb = cmul(bb, rb);
    // W = A' + j B', conjugated (the inverse runs forward) and scaled by g / N
    w[i] = make_float2(g * (pa.x - pb.y), -g * (pa.y + pb.x));
  }
  dft16(w);   // the inverse's first pass: its inputs j + r T are this lane's bins
  __syncthreads();
  {
    const int p0 = fpad(16 * j);
#pragma unroll
    for (int r = 0; r < 16; r++) lds[p0 + r] = w[r];
  }
  __syncthreads();
  float xa[16], xb[16];
  fft_passes<FN, 16, false>(lds, J.twid, PairOut{xa, xb});
#pragma unroll
  for (int x = 0; x < 2; x++) {
#pragma unroll
    for (int i = FGUARD / FT; i < (FGUARD + FHOP) / FT; i++) {
      const int64_t t = F[x] + j + FT * i;
      if (t < n) gptr(J.xr)[t] = x ? xb[i] : xa[i];
    }
  }
}

void rx_launch_pamfd(int stage, const RxLaunch &L, int64_t maxn, hipStream_t s) {
  const unsigned cnt = (unsigned)L.count;
  const int64_t npair = (maxn + 2 * FHOP - 1) / (2 * FHOP);
  if (stage == ST_PAM_MF) hipLaunchKernelGGL(pamfd_eq, dim3((unsigned)npair, cnt), dim3(FT), 0, s, L);
  else hipLaunchKernelGGL(pamfd_clock, dim3((unsigned)npair, cnt), dim3(FT), 0, s, L);
}

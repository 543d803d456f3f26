// Equaliser tail of both chains: prefix adaptation (one wavefront per
// buffer), block-parallel DD-LMS FFE (one lane pair per block; the paper
// runs the 8192 blocks of a buffer in parallel, Sec. 2, second paragraph),
// decisions, Gray demapping, bit packing and error counting (Sec. 3, second
// paragraph).
#include <type_traits>

#include "rx_dev.hpp"

// Serial adaptive filters of the prefix stage, one wavefront: lane l holds
// tap t = l mod 32 (zero beyond K); lanes 0..31 form the real parts of the
// products w_t x_t, lanes 32..63 the imaginary parts, so one reduction
// within each half gives Re z (lane 31) and Im z (lane 63): DPP within rows
// of 16 (quad swaps, half-row and row mirrors), then row_bcast:15 adds row 0
// into row 1 and row 2 into row 3.
#define DPP(v, ctrl, rm) __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, rm, 0xF, false))
__device__ __forceinline__ float2 split_sum(float v) {
  v += DPP(v, 0xB1, 0xF);    // quad_perm [1,0,3,2]
  v += DPP(v, 0x4E, 0xF);    // quad_perm [2,3,0,1]
  v += DPP(v, 0x141, 0xF);   // row_half_mirror
  v += DPP(v, 0x140, 0xF);   // row_mirror
  v += DPP(v, 0x142, 0xA);   // row_bcast:15 into rows 1 and 3
  return make_float2(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 31)),
                     __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)));
}
#undef DPP

// The value of the other lane of an even/odd lane pair (DPP quad_perm [1,0,3,2]).
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// One lane's view of the input sample of its tap: products w x split by half.
struct PfxLane {
  bool hi;    // lane >= 32: imaginary part of the product
  __device__ float part(float2 w, float2 x) const {
    // lanes 0..31: wr xr - wi xi; lanes 32..63: wr xi + wi xr
    const float xa = hi ? x.y : x.x, xb = hi ? x.x : -x.y;
    return fmaf(w.y, xb, w.x * xa);
  }
};

#define PFX_OFF (2 * RX_LAG + RX_KMAX / 2)
#define PFX_UL (2 * RX_PREFIX_MAX + 2 * RX_LAG + 2 * PFX_OFF)

#define PFX_T 1024
// Prefix stage, one workgroup per buffer.  The serial loops run on one
// wavefront; the workgroup holds a CU anyway (its LDS), so it brings
// PFX_T / 64 wavefronts to the parallel parts (AGC sums, the sample window,
// the candidate-delay outputs and correlations), which are latency-bound.
//  KK : CMA over the prefix (centre-tap start), static Viterbi-Viterbi phase
//       of the last 2048 CMA outputs, taps rotated and scaled to odd-integer
//       units;
//  both: delay search over [-64, 64] symbols on the known prefix (KK also
//       picks the quadrant), then data-aided LMS over the prefix -> w0.
__global__ __launch_bounds__(PFX_T) void rx_prefix(RxLaunch L) {
  __shared__ float2 u[PFX_UL];
  __shared__ float2 zp[RX_PREFIX_MAX + 2 * RX_LAG];
  __shared__ float2 ar[RX_PREFIX_MAX];
  __shared__ float2 cs[2 * RX_LAG + 1];
  __shared__ float2 w[RX_KMAX];
  __shared__ double red[PFX_T / 64];
  __shared__ int sel[2];
  __shared__ float th0s;

  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int kk = J.kk, K = J.ffe_taps, c = (K - 1) / 2, P = J.prefix;
  const int64_t nx = kk ? n / 2 : n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

  // KK: carrier mean and AGC gain from the front end's per-workgroup sums:
  // sum |Z - m T|^2 = sum|Z|^2 - 2 Re(conj(m) sum Z conj(T)) + |m|^2 sum|T|^2.
  // The PAM samples arrive already scaled.
  float g = 1.0f;
  float2 mean = make_float2(0.0f, 0.0f);
  if (kk) {
    const int64_t npairs = ((n + J.hop - 1) / J.hop + 1) / 2;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = threadIdx.x; i < npairs; i += PFX_T) {
      const double2 a = J.part[3 * i], b = J.part[3 * i + 1], c2 = J.part[3 * i + 2];
      v[0] += a.x; v[1] += a.y; v[2] += b.x; v[3] += b.y; v[4] += c2.x; v[5] += c2.y;
    }
    for (int q = 0; q < 6; q++) v[q] = block_sum(v[q], red);
    const double mr = v[0] / (double)n, mi = v[1] / (double)n;
    const double pw = v[2] - 2.0 * (mr * v[4] + mi * v[5]) + (mr * mr + mi * mi) * v[3];
    const double gd = 1.0 / sqrt(pw / (double)nx);
    g = (float)gd;
    mean = make_float2((float)mr, (float)mi);
    if (threadIdx.x == 0) {
      J.sc->agc = gd;
      J.sc->mean_re = mr;
      J.sc->mean_im = mi;
    }
  }
  const auto zin = gview(J.z);
  const auto xin = gptr(J.xr);
#pragma unroll 8
  for (int idx = threadIdx.x; idx < PFX_UL; idx += PFX_T) {
    const int64_t j = (int64_t)idx - PFX_OFF;
    float2 v = make_float2(0.0f, 0.0f);
    if (j >= 0 && j < nx) v = kk ? kk_sample(J, zin, j, n, mean, g, 0) : make_float2(xin[j], 0.0f);
    u[idx] = v;
  }
  for (int k = threadIdx.x; k < P; k += PFX_T) ar[k] = ref_symbol(J, k);
  __syncthreads();

  const int tap = lane & 31;
  const PfxLane pl{lane >= 32};
  // LDS slot of this lane's input at step k: u[PFX_OFF + 2 k + c - tap]; taps
  // beyond K read slot 0, which holds a zero (a sample before the buffer)
  const int xbase = tap < K ? PFX_OFF + c - tap : 0, xstep = tap < K ? 2 : 0;
  if (wv == 0) {
    float2 wi = make_float2(0.0f, 0.0f);
    if (tap == c) wi.x = kk ? 1.0f : J.ea2_sqrt;
    float th0 = 0.0f;
    if (kk) {
      // CMA: e = mu (R2 - |z|^2) z, w += e conj(x); static Viterbi-Viterbi
      // sum of z^4 over the last 2048 outputs
      float s4r = 0.0f, s4i = 0.0f;
      const float mur2 = J.mu_cma * J.r2, mu = J.mu_cma;
      float2 xn = u[xbase];
      auto cma_step = [&](int k, bool vv) {
        const float2 xi = xn;
        xn = u[xbase + xstep * (k + 1)];   // in range: u extends past the prefix
        const float2 z = split_sum(pl.part(wi, xi));
        if (vv) {
          const float ar2 = z.x * z.x - z.y * z.y, ai2 = 2.0f * z.x * z.y;
          s4r += ar2 * ar2 - ai2 * ai2;
          s4i += 2.0f * ar2 * ai2;
        }
        const float f = fmaf(-mu, fmaf(z.y, z.y, z.x * z.x), mur2);
        const float er = z.x * f, ei = z.y * f;
        wi.x = fmaf(er, xi.x, fmaf(ei, xi.y, wi.x));
        wi.y = fmaf(ei, xi.x, fmaf(-er, xi.y, wi.y));
      };
      const int k1 = P > 2048 ? P - 2048 : 0;
      for (int k = 0; k < k1; k++) cma_step(k, false);
      for (int k = k1; k < P; k++) cma_step(k, true);
      th0 = 0.25f * atan2f(-s4i, -s4r);
      float sn, cn;
      sincosf(-th0, &sn, &cn);
      wi = cscale(cmul(wi, make_float2(cn, sn)), J.ea2_sqrt);
    }
    if (lane < RX_KMAX) w[lane] = lane < K ? wi : make_float2(0.0f, 0.0f);
    if (lane == 0) th0s = th0;
  }
  __syncthreads();

  // FFE outputs with the start taps for every candidate delay
  for (int jj = threadIdx.x; jj < P + 2 * RX_LAG; jj += PFX_T) {
    const int j = jj - RX_LAG;
    float2 z = make_float2(0.0f, 0.0f);
    for (int i = 0; i < K; i++) z = cadd(z, cmul(w[i], u[PFX_OFF + 2 * j + c - i]));
    zp[jj] = z;
  }
  __syncthreads();
  // correlation with the known prefix, candidates in preference order
  // s = 0, -1, 1, -2, 2, ...
  for (int t = wv; t <= 2 * RX_LAG; t += PFX_T / 64) {
    const int s = (t == 0) ? 0 : ((t & 1) ? -((t + 1) / 2) : t / 2);
    float cr = 0.0f, ci = 0.0f;
    for (int k = lane; k < P; k += 64) {
      const float2 p = cmulc(zp[k + s + RX_LAG], ar[k]);
      cr += p.x;
      ci += p.y;
    }
    cr = wave_sum(cr);
    ci = wave_sum(ci);
    if (lane == 0) cs[t] = make_float2(cr, ci);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float best = -INFINITY;
    int bt = 0;
    for (int t = 0; t <= 2 * RX_LAG; t++) {
      const float2 v = cs[t];
      const float sc = kk ? (v.x * v.x + v.y * v.y) : v.x;
      if (sc > best) { best = sc; bt = t; }
    }
    const int s = (bt == 0) ? 0 : ((bt & 1) ? -((bt + 1) / 2) : bt / 2);
    int q = 0;
    if (kk) {
      const float2 v = cs[bt];
      const int qq = (int)lrintf(-atan2f(v.y, v.x) / 1.5707963267948966f);
      q = ((qq % 4) + 4) % 4;
    }
    sel[0] = s;
    sel[1] = q;
  }
  __syncthreads();

  if (wv == 0) {
    // data-aided LMS over the prefix at the chosen delay: e = mu (a - z)
    const int s = sel[0], q = sel[1];
    float2 wi = tap < K ? w[tap] : make_float2(0.0f, 0.0f);
    const float2 jq = q == 0 ? make_float2(1, 0) : q == 1 ? make_float2(0, 1) : q == 2 ? make_float2(-1, 0) : make_float2(0, -1);
    wi = cmul(wi, jq);
    const float mu = J.mu;
    const int xb2 = tap < K ? xbase + 2 * s : 0;
    float2 xn = u[xb2];
    float2 an = ar[0];
    for (int k = 0; k < P; k++) {
      const float2 xi = xn, a = an;   // next step's input and symbol read one step ahead
      xn = u[xb2 + xstep * (k + 1)];
      an = ar[k + 1 < P ? k + 1 : k];
      const float2 z = split_sum(pl.part(wi, xi));
      const float er = mu * (a.x - z.x), ei = mu * (a.y - z.y);
      wi.x = fmaf(er, xi.x, fmaf(ei, xi.y, wi.x));
      wi.y = fmaf(ei, xi.x, fmaf(-er, xi.y, wi.y));
    }
    if (lane < RX_KMAX) J.sc->w0[lane] = lane < K ? wi : make_float2(0.0f, 0.0f);
    if (lane == 0) {
      J.sc->lag = s;
      J.sc->rot = q;
      J.sc->theta0 = th0s;
      J.sc->fallback = 0;
    }
  }
}

// Block-parallel DD-LMS: each block of `blk` symbols is adapted from w0
// independently (a decision feedback error cannot leave its block).  A block
// runs on a lane pair split by polyphase: at 2 samples per symbol tap i of the
// FFE meets only samples of the parity of i, so lane h of the pair holds the
// taps i = 2a + h and every other sample, xe[j] = x[2j - h]; tap a of either
// lane sees xe[kk + C - a] at step kk, and one DPP swap adds the two partial
// outputs.  Half the taps and half the window per lane keep the kernel at
// four wavefronts per SIMD.  Block streams are 2*blk samples apart, so they
// are staged through LDS in chunks of BC steps: the workgroup loads every
// block's next 2*BC samples with coalesced reads (all issued before any is
// used), each lane runs BC steps from registers, and the soft outputs go
// back out the same way.  (Five wavefronts per SIMD, with 4-step chunks, is
// faster alone but slows the chain: its workgroups keep the front end off
// more CUs.)
template <bool CPLX, int K, int BC>   // BC: steps per staged chunk (a tuned choice)
__global__ __launch_bounds__(256) void rx_blocks(RxLaunch L) {
  using T = typename std::conditional<CPLX, float2, float>::type;
  constexpr int NBW = 128;   // blocks per workgroup (one lane pair each)
  __shared__ T sin_[NBW * (2 * BC + 1)];
  __shared__ T sout[NBW * (BC + 1)];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int64_t nx = CPLX ? n / 2 : n;
  const int blk = J.blk;
  const int64_t nsym = n / (CPLX ? 4 : 2);
  const int64_t nb = nsym / blk;
  const int64_t b0 = (int64_t)blockIdx.x * NBW;
  if (b0 >= nb) return;
  if (J.mlp && !J.sc->fallback) return;   // the learned equaliser's output stands
  const int lb = threadIdx.x >> 1, h = threadIdx.x & 1;
  const int64_t b = b0 + lb;
  const bool active = b < nb;
  constexpr int C = (K - 1) / 2;
  const float mu = J.mu;
  const int m = J.m_axis;
  const float g = CPLX ? (float)J.sc->agc : 1.0f;
  const float2 mean = make_float2((float)J.sc->mean_re, (float)J.sc->mean_im);
  const int s = J.sc->lag;
  const int64_t g0 = L.s0[jb] > 0 ? L.s0[jb] : 0;   // stream index of sample 0 (downshift phase)
  const auto zin = gview(J.z);
  const auto xin = gptr(J.xr);
  float2 *const soft = J.soft;
  auto load = [&](int64_t j) -> T {
    if constexpr (CPLX) {
      return kk_sample<true>(J, zin, j, n, mean, g, g0);
    } else {
      return (j >= 0 && j < nx) ? xin[j] : 0.0f;
    }
  };
  constexpr int LPP = 256 / (2 * BC);          // blocks staged per pass of the workgroup
  static_assert(256 % (2 * BC) == 0 && NBW % LPP == 0 && (NBW * 2 * BC) % 256 == 0, "staging assumes whole blocks per pass");
  const float2 Mc = cscale(cmul(mean, J.c0), g);
  const float2 rstep = cis_rev(-downshift_rev(J.r, 2 * 2 * LPP * (int64_t)blk));
  // taps 2a + h; lane 1's extra tap a = C (index K) stays zero: its update is masked
  float2 w[C + 1];
#pragma unroll
  for (int a = 0; a <= C; a++) w[a] = (2 * a + h < K) ? J.sc->w0[2 * a + h] : make_float2(0.0f, 0.0f);
  // lane h's last tap, 2 C + h, exists for lane 0 always and for lane 1 only
  // with an even tap count (the paper's 4 taps)
  const float umask = 2 * C + h < K ? 1.0f : 0.0f;
  T xe[C + 1 + BC];   // xe[j] = sample p0 - C + 2 j - h (+ 2 BC per chunk)
  const int64_t p0 = 2 * (b * blk + s);
  {
    // start window: all reads first (index clamped), then formed; samples
    // outside the interior are recomputed exactly
    T xr0[C + 1];
#pragma unroll
    for (int j = 0; j <= C; j++) {
      const int64_t pj = p0 - C + 2 * j - h;
      if constexpr (CPLX) xr0[j] = zin[pj < 0 ? 0 : (pj >= nx ? nx - 1 : pj)];
      else xr0[j] = xin[pj < 0 ? 0 : (pj >= nx ? nx - 1 : pj)];
    }
    bool edge = false;
    // carrier phasor P(p) = exp(-j 2 pi frac(2 r p)) at p = p0 - C - h, then
    // one fixed rotation per step of two samples
    float2 P = make_float2(1.0f, 0.0f), r4 = P;
    if constexpr (CPLX) {
      P = cis_rev(-downshift_rev(J.r, g0 + 2 * (p0 - C - h)));
      r4 = cis_rev(-downshift_rev(J.r, 4));
    }
#pragma unroll
    for (int j = 0; j <= C; j++) {
      const int64_t pj = p0 - C + 2 * j - h;
      if constexpr (CPLX) {
        edge |= !kk_interior(pj, n);
        xe[j] = csub(cscale(xr0[j], g), cmul(Mc, P));
        P = cmul(P, r4);
      } else {
        xe[j] = (pj >= 0 && pj < nx) ? xr0[j] : 0.0f;
      }
    }
    if (CPLX && edge) {   // a block at a buffer end
#pragma unroll
      for (int j = 0; j <= C; j++) {
        const int64_t pj = p0 - C + 2 * j - h;
        if (!kk_interior(pj, n)) xe[j] = load(pj);
      }
    }
  }
  float s4r = 0.0f, s4i = 0.0f;
  const int nch = blk / BC;
  for (int ch = 0; ch < nch; ch++) {
    // block l's next 2*BC samples start at p0_l + C + 1 + 2*BC*ch
    if constexpr (CPLX) {
      // thread: stream position jj of blocks l0 + LPP i, whose samples are
      // 2 LPP blk apart, so the carrier phasor P(p) = exp(-j 2 pi frac(2 r p))
      // advances by one fixed rotation from an FP64 anchor per chunk; the
      // interior sample is then u = g z - (g mean c0) P (the edge samples
      // take the exact form).
      const int l0 = threadIdx.x / (2 * BC), jj = threadIdx.x % (2 * BC);
      const int64_t pa = 2 * ((b0 + l0) * blk + s) + C + 1 + 2 * BC * ch + jj;
      // all reads first (index clamped into the stream) so their latencies
      // overlap; samples outside the interior are recomputed exactly
      float2 zr[NBW / LPP];
#pragma unroll
      for (int i = 0; i < NBW / LPP; i++) {
        const int64_t pl = pa + (int64_t)i * 2 * LPP * blk;
        zr[i] = zin[pl < 0 ? 0 : (pl >= nx ? nx - 1 : pl)];
      }
      float2 P = cis_rev(-downshift_rev(J.r, g0 + 2 * pa));
      bool edge = false;
#pragma unroll
      for (int i = 0; i < NBW / LPP; i++) {
        const int64_t pl = pa + (int64_t)i * 2 * LPP * blk;
        edge |= !(pl >= 16 && 2 * pl + 32 < n);
        sin_[(l0 + LPP * i) * (2 * BC + 1) + jj] = csub(cscale(zr[i], g), cmul(Mc, P));
        P = cmul(P, rstep);
      }
      if (edge) {   // the few samples near the buffer ends, exact
#pragma unroll 1
        for (int i = 0; i < NBW / LPP; i++) {
          const int64_t pl = pa + (int64_t)i * 2 * LPP * blk;
          if (!(pl >= 16 && 2 * pl + 32 < n)) sin_[(l0 + LPP * i) * (2 * BC + 1) + jj] = load(pl);
        }
      }
    } else {
      constexpr int NE = NBW * 2 * BC / 256;
      float xr[NE];
#pragma unroll
      for (int i = 0; i < NE; i++) {   // all reads first, index clamped into the stream
        const int e = threadIdx.x + 256 * i;
        const int64_t pl = 2 * ((b0 + e / (2 * BC)) * blk + s) + C + 1 + 2 * BC * ch + e % (2 * BC);
        xr[i] = xin[pl < 0 ? 0 : (pl >= nx ? nx - 1 : pl)];
      }
#pragma unroll
      for (int i = 0; i < NE; i++) {
        const int e = threadIdx.x + 256 * i;
        const int l = e / (2 * BC), jj = e % (2 * BC);
        const int64_t pl = 2 * ((b0 + l) * blk + s) + C + 1 + 2 * BC * ch + jj;
        sin_[l * (2 * BC + 1) + jj] = (pl >= 0 && pl < nx) ? xr[i] : 0.0f;
      }
    }
    __syncthreads();
    // xe[C + 1 + t] = staged position 2 t + 1 - h of this block
#pragma unroll
    for (int t = 0; t < BC; t++) xe[C + 1 + t] = sin_[lb * (2 * BC + 1) + 2 * t + 1 - h];
#pragma unroll
    for (int kk = 0; kk < BC; kk++) {
      if constexpr (CPLX) {
        // z = sum_i w_i x_i and w_i += e conj(x_i), four FMAs per tap each;
        // the dot product in two interleaved partial sums per component (even
        // and odd a) so four independent FMA chains are in flight
        float2 z0 = make_float2(0.0f, 0.0f), z1 = z0;
#pragma unroll
        for (int a = 0; a <= C; a++) {
          const float2 xv = xe[kk + C - a];
          float2 &zz = (a & 1) ? z1 : z0;
          zz.x = fmaf(w[a].x, xv.x, zz.x);
          zz.x = fmaf(-w[a].y, xv.y, zz.x);
          zz.y = fmaf(w[a].x, xv.y, zz.y);
          zz.y = fmaf(w[a].y, xv.x, zz.y);
        }
        float2 z = cadd(z0, z1);
        z.x += pair_swap(z.x);
        z.y += pair_swap(z.y);
        const float2 e = make_float2(mu * (decide_level(z.x, m) - z.x), mu * (decide_level(z.y, m) - z.y));
#pragma unroll
        for (int a = 0; a <= C; a++) {
          const float2 xv = xe[kk + C - a];
          const float2 ea = a == C ? cscale(e, umask) : e;
          w[a].x = fmaf(ea.x, xv.x, w[a].x);
          w[a].x = fmaf(ea.y, xv.y, w[a].x);
          w[a].y = fmaf(ea.y, xv.x, w[a].y);
          w[a].y = fmaf(-ea.x, xv.y, w[a].y);
        }
        const float a2 = z.x * z.x - z.y * z.y, b2 = 2.0f * z.x * z.y;
        s4r += a2 * a2 - b2 * b2;
        s4i += 2.0f * a2 * b2;
        if (h == 0) sout[lb * (BC + 1) + kk] = z;
      } else {
        float z = 0.0f;
#pragma unroll
        for (int a = 0; a <= C; a++) z = fmaf(w[a].x, xe[kk + C - a], z);
        z += pair_swap(z);
        const float e = mu * (decide_level(z, m) - z);
#pragma unroll
        for (int a = 0; a <= C; a++) w[a].x = fmaf(a == C ? e * umask : e, xe[kk + C - a], w[a].x);
        if (h == 0) sout[lb * (BC + 1) + kk] = z;
      }
    }
#pragma unroll
    for (int j = 0; j <= C; j++) xe[j] = xe[j + BC];
    __syncthreads();
    for (int e = threadIdx.x; e < NBW * BC; e += 256) {
      const int l = e / BC, kk = e % BC;
      if (b0 + l < nb) {
        const T v = sout[l * (BC + 1) + kk];
        if constexpr (CPLX) gstore(soft, (b0 + l) * blk + BC * ch + kk, v);
        else gptr(reinterpret_cast<float *>(soft))[(b0 + l) * blk + BC * ch + kk] = v;   // PAM: real soft symbols
      }
    }
  }
  if (CPLX && active && h == 0) gstore(J.s4, b, make_float2(s4r, s4i));
}

// Precision form of the FFE (KK): the prefix taps w0 frozen for the buffer
// and applied as a Toeplitz GEMM on MFMA with narrow operands and FP32
// accumulation.  A row = [Re x | Im x] of the 64-sample window of a tile of
// 16 symbols (x = AGC'd 2-sps samples from 2(k0+s)-C), B = [[Wr, Wi],
// [-Wi, Wr]] with W[t][q] = w0[2C + 2q - t]; 4 K-steps x 2 column tiles.
// A group is 16 tiles (256 symbols = two VV blocks), whose z^4 sums the
// wavefront also forms; each wavefront takes GPW consecutive groups (a tuned choice)
// (the next group's window in flight while the current one is filtered),
// and the B fragments are built once per workgroup, in LDS.
#define FFE_PL 672   // staged plane length: window positions 0..543 with 8 elements of padding per 32
// LDS index of window position t: the 16-byte A reads of the 16 rows then
// fall on distinct banks (row stride 20 dwords)
__device__ __forceinline__ int ffe_idx(int t) { return t + ((t >> 5) << 3); }
template <int PREC, int GPW>
__global__ __launch_bounds__(256) void rx_ffe_mfma(RxLaunch L) {
  using NT = NarrowT<PREC>;
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb], nx = n / 2, nsym = n / 4;
  const int lane = threadIdx.x & 63;
  const int64_t grp0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * GPW;
  const int K = J.ffe_taps, C = (K - 1) / 2;
  const int row = lane & 15, kq = lane >> 4;
  // B fragments, shared by the workgroup's wavefronts in LDS (wavefront ks
  // builds step ks): kk = 32 ks + 8 kq + j (t = kk % 64, part = kk / 64),
  // column q = row of output tile ct (0: Re z, 1: Im z)
  __shared__ __align__(16) typename NT::vec bl[8][64];
  {
    const int ks = threadIdx.x >> 6;
    typename NT::vec b0, b1;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int kk = 32 * ks + 8 * kq + j, t = kk & 63, part = kk >> 6;
      const int i = 2 * C + 2 * row - t;
      float2 w = make_float2(0.0f, 0.0f);
      if (i >= 0 && i < K) w = J.sc->w0[i];
      const float wr = NT::cvt(w.x), wi = NT::cvt(w.y);   // operands rounded once
      b0[j] = NT::cvt(part == 0 ? wr : -wi);
      b1[j] = NT::cvt(part == 0 ? wi : wr);
    }
    bl[2 * ks][lane] = b0;
    bl[2 * ks + 1][lane] = b1;
  }
  __syncthreads();
  if (grp0 * 256 >= nsym) return;
  const int s = J.sc->lag;
  const float g = (float)J.sc->agc;
  const float2 mean = make_float2((float)J.sc->mean_re, (float)J.sc->mean_im);
  const int64_t g0 = L.s0[jb] > 0 ? L.s0[jb] : 0;   // stream index of sample 0 (downshift phase)
  const auto zin = gview(J.z);
  // The group's 16 windows cover samples base0 .. base0 + 543; they are
  // staged once per group into this wavefront's LDS planes as u rounded to
  // the narrow type, from coalesced 16-byte loads (pairs of samples from the
  // even index R0 = base0 - (base0 mod 2)).  Interior samples u = g z - (g mean c0) P,
  // P(p) = exp(-j 2 pi frac(2 r p)): one FP64 anchor per lane and group, then
  // fixed rotations; edge samples take the exact form.
  __shared__ __align__(16) typename NT::elem ul[4][2 * FFE_PL];
  typename NT::elem *const ure = ul[threadIdx.x >> 6], *const uim = ure + FFE_PL;
  const float2 Mc = cscale(cmul(mean, J.c0), g);
  const float2 r1 = cis_rev(-downshift_rev(J.r, 2));
  const float2 r128 = cis_rev(-downshift_rev(J.r, 2 * 128));
  // window pairs of group grp (index clamped into the buffer; pairs outside
  // the interior are recomputed exactly below)
  auto load_pairs = [&](int64_t grp, float4 (&zz)[5]) {
    const int64_t base0 = 2 * (grp * 256 + s) - C;
    const int64_t R0 = base0 - (base0 & 1);
#pragma unroll
    for (int it = 0; it < 5; it++) {
      const int64_t p = R0 + 2 * (lane + 64 * it);
      zz[it] = gload4(J.z, (p < 0 ? 0 : (p > nx - 2 ? nx - 2 : p)) >> 1);
    }
  };
  float4 zn[5];
  load_pairs(grp0, zn);
  for (int gi = 0; gi < GPW; gi++) {
    const int64_t grp = grp0 + gi;
    if (grp * 256 >= nsym) break;
    float4 zc[5];
#pragma unroll
    for (int it = 0; it < 5; it++) zc[it] = zn[it];
    if (gi + 1 < GPW && (grp + 1) * 256 < nsym) load_pairs(grp + 1, zn);   // in flight during this group
    const int64_t base0 = 2 * (grp * 256 + s) - C;
    const int odd = (int)(base0 & 1);
    const int64_t R0 = base0 - odd;
    float2 P = cis_rev(-downshift_rev(J.r, g0 + 2 * (R0 + 2 * lane)));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // the previous group's reads are done
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int it = 0; it < 5; it++) {
      const int pi = lane + 64 * it;   // pair pi: samples R0 + 2 pi, R0 + 2 pi + 1
      if (pi < 273) {
        const int64_t p = R0 + 2 * pi;
        float2 u0, u1;
        if (p >= 16 && 2 * (p + 1) + 32 < n) {
          const float4 zz = zc[it];
          u0 = csub(cscale(make_float2(zz.x, zz.y), g), cmul(Mc, P));
          u1 = csub(cscale(make_float2(zz.z, zz.w), g), cmul(Mc, cmul(P, r1)));
        } else {
          u0 = kk_sample(J, zin, p, n, mean, g, g0);
          u1 = kk_sample(J, zin, p + 1, n, mean, g, g0);
        }
        const int t0 = 2 * pi - odd;   // window position of sample p
        if (t0 >= 0 && t0 < 544) {
          ure[ffe_idx(t0)] = NT::cvt(u0.x);
          uim[ffe_idx(t0)] = NT::cvt(u0.y);
        }
        if (t0 + 1 < 544) {
          ure[ffe_idx(t0 + 1)] = NT::cvt(u1.x);
          uim[ffe_idx(t0 + 1)] = NT::cvt(u1.y);
        }
      }
      P = cmul(P, r128);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // staged planes visible to the wavefront
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    rx_f32x4 zr = {0.0f, 0.0f, 0.0f, 0.0f}, zi = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 4; ks++) {
      // A[row][8 kq + j] = window sample 32 row + 32 (ks % 2) + 8 kq + j
      const typename NT::elem *pl = ks < 2 ? ure : uim;
      const typename NT::vec a = *reinterpret_cast<const typename NT::vec *>(pl + ffe_idx(32 * row + 32 * (ks & 1) + 8 * kq));
      zr = NT::mfma(a, bl[2 * ks][lane], zr);
      zi = NT::mfma(a, bl[2 * ks + 1][lane], zi);
    }
    float s4r = 0.0f, s4i = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int64_t k = (grp * 16 + 4 * kq + j) * 16 + row;
      const float2 z = make_float2(zr[j], zi[j]);
      gstore(J.soft, k, z);
      const float a2 = z.x * z.x - z.y * z.y, b2 = 2.0f * z.x * z.y;
      s4r += a2 * a2 - b2 * b2;
      s4i += 2.0f * a2 * b2;
    }
    // lanes 0..31 hold tiles 0..7 (block 2 grp), lanes 32..63 tiles 8..15
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      s4r += __shfl_xor(s4r, o, 64);
      s4i += __shfl_xor(s4i, o, 64);
    }
    if ((lane & 31) == 0) gstore(J.s4, 2 * grp + (lane >> 5), make_float2(s4r, s4i));
  }
}

// Decisions, Gray demapping, packing and error counting: eight consecutive
// symbols per lane (one derotation phase, one 8*bps-bit chunk of the stream);
// the workgroup's DEC_SYMS symbols are packed in LDS, written out as whole
// words, and its error counts added with one set of atomics.
template <int DEC_SYMS>   // symbols per workgroup, 8 per thread (a tuned choice)
__global__ __launch_bounds__(DEC_SYMS / 8) void rx_decide(RxLaunch L) {
  constexpr int NT = DEC_SYMS / 8;
  __shared__ uint32_t wb[DEC_SYMS * 4 / 32];   // the workgroup's packed bits (up to 4 per symbol)
  __shared__ uint32_t red[NT / 64];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int kk = J.kk, bps = J.bps, m = J.m_axis, P = J.prefix;
  const int64_t nsym = n / (kk ? 4 : 2);
  const int64_t kbase = (int64_t)blockIdx.x * DEC_SYMS;
  if (kbase >= nsym) return;   // nsym is a multiple of 256
  // emitted symbols [k_lo, k_hi) of this input (all of an independent
  // buffer; a stream buffer holds its last samples back and, after the
  // first, skips the prepended ones), output bit 0 = symbol k_lo; the
  // stream's symbol index is kg0 + k
  const RxSpan sp = rx_span(J, n, L.s0[jb]);
  const auto out = gptr(reinterpret_cast<uint32_t *>(L.bits[jb]));
  float2 *const soft = J.soft;
  const int nw = DEC_SYMS * bps / 32;
  if (bps != 4)   // 4 bits per symbol: each thread's 8 symbols are one whole output word (below)
    for (int i = threadIdx.x; i < nw; i += NT) wb[i] = 0u;
  // this thread: symbols k0 .. k0 + 7 (one DD-LMS block, so one phase); the
  // emission bounds are multiples of 256 symbols, so a thread's 8 are all in
  // or all out
  const int64_t k0 = kbase + 8 * threadIdx.x;
  const bool valid = k0 < nsym;   // then k0 + 8 <= nsym
  const bool emit = valid && k0 >= sp.k_lo && k0 < sp.k_hi;
  // counted symbols, symbol errors and bit errors of this thread, packed as
  // cs | se << 10 | be << 20: a wavefront counts at most 512 symbols and
  // 2048 bit errors (4 bits per symbol at most), so no field overflows
  uint32_t cnt = 0;
  uint32_t chunk = 0;   // symbol k0 + i at bits [bps i, bps (i + 1)), MSB of the symbol first
  if (emit) {
    // counted symbols of this thread: i in [ilo, ihi) (stream indices from
    // P + 64 on; an independent buffer also leaves its last 64 out)
    const int64_t clo = P + RX_GUARD - sp.kg0, chi = J.stream ? sp.k_hi : nsym - RX_GUARD;
    const int64_t lo64 = clo - k0, hi64 = chi - k0;
    const int ilo = (int)(lo64 < 0 ? 0 : (lo64 > 8 ? 8 : lo64)), ihi = (int)(hi64 < 0 ? 0 : (hi64 > 8 ? 8 : hi64));
    // the thread's reference symbols, packed like the output: from the
    // handle's stream of them (bits [bps k0, bps (k0 + 8)): k0 is a
    // multiple of 8, so they start at bit (bps k0) mod 32 of a word and end
    // within the next), or, for a stream, from the seed at the stream index
    uint32_t refc = 0u;
    if (J.stream) {
#pragma unroll
      for (int i = 0; i < 8; i++)
        refc |= (__builtin_bitreverse32(ref_seed_bits(J, sp.kg0 + k0 + i)) >> (32 - bps)) << (bps * i);
    } else {
      const int64_t ob = (int64_t)bps * k0;
      const auto rw = gptr(J.refw);
      // the second word only where the 8 bps bits cross into it: then it still
      // holds bits of these symbols, so no read goes past the stream's last word
      const uint64_t w1 = ((ob & 31) + 8 * bps > 32) ? (uint64_t)rw[(ob >> 5) + 1] : 0ull;
      refc = (uint32_t)(((uint64_t)rw[ob >> 5] | (w1 << 32)) >> (ob & 31));
    }
    float2 zv[8];
    if (kk) {   // complex soft symbols
#pragma unroll
      for (int h = 0; h < 4; h++) {
        const float4 q = gload4(soft + k0, h);
        zv[2 * h] = make_float2(q.x, q.y);
        zv[2 * h + 1] = make_float2(q.z, q.w);
      }
    } else {    // PAM: real soft symbols, packed
      const float *const sr = reinterpret_cast<const float *>(soft) + k0;
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const float4 q = gload4(sr, h);
        zv[4 * h] = make_float2(q.x, 0.0f);
        zv[4 * h + 1] = make_float2(q.y, 0.0f);
        zv[4 * h + 2] = make_float2(q.z, 0.0f);
        zv[4 * h + 3] = make_float2(q.w, 0.0f);
      }
    }
    const float2 rot = kk ? cis_rev(-gptr(J.theta)[k0 / J.blk] * 0.15915494309189535f) : make_float2(1.0f, 0.0f);
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const int64_t k = k0 + i;
      uint32_t sym;
      if (kk) {
        const float2 z = cmul(zv[i], rot);
        if (J.debug) gstore(soft, k, z);
        const uint32_t gi = (uint32_t)decide_index(z.x, m), gq = (uint32_t)decide_index(z.y, m);
        sym = ((gi ^ (gi >> 1)) << (bps >> 1)) | (gq ^ (gq >> 1));
      } else {
        const uint32_t gi = (uint32_t)decide_index(zv[i].x, m);
        sym = gi ^ (gi >> 1);
      }
      chunk |= (__builtin_bitreverse32(sym) >> (32 - bps)) << (bps * i);
    }
    const uint32_t x = chunk ^ refc;   // differing bits, symbol i at [bps i, bps (i + 1))
#pragma unroll
    for (int i = 0; i < 8; i++) {
      if (i >= ilo && i < ihi) {
        const uint32_t ne = (uint32_t)__popc((x >> (bps * i)) & ((1u << bps) - 1u));
        cnt += 1u + ((ne > 0u) << 10) + (ne << 20);
      }
    }
  }
  if (bps == 4) {   // (uniform) symbols k0 .. k0 + 7 are exactly output word (k0 - k_lo) / 8
    if (emit) out[(k0 - sp.k_lo) / 8] = chunk;
  } else {          // the workgroup's words assembled in LDS, then written whole
    __syncthreads();
    if (emit) {
      const int lb = 8 * bps * threadIdx.x, wi = lb >> 5, off = lb & 31;
      atomicOr(&wb[wi], chunk << off);
      if (off + 8 * bps > 32) atomicOr(&wb[wi + 1], chunk >> (32 - off));
    }
    __syncthreads();
    // word i holds bits of symbols from kbase + 32 i / bps on; the emission
    // bounds are multiples of 256 symbols, i.e. of whole words
    const int64_t nsw = (nsym - kbase < DEC_SYMS ? nsym - kbase : DEC_SYMS) * bps / 32;
    const int64_t wlo = (sp.k_lo - kbase) * bps / 32, whi = (sp.k_hi - kbase) * bps / 32;
    for (int i = threadIdx.x; i < nsw; i += NT)
      if (i >= wlo && i < whi) out[(kbase - sp.k_lo) * bps / 32 + i] = wb[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long cs = 0, se = 0, be = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) {
      cs += red[w] & 1023u;
      se += (red[w] >> 10) & 1023u;
      be += red[w] >> 20;
    }
    if (cs) {
      atomicAdd(&J.sc->stats[1], cs);
      atomicAdd(&J.sc->stats[2], cs * (unsigned long long)bps);
      atomicAdd(&J.sc->stats[3], be);
      atomicAdd(&J.sc->stats[4], se);
    }
    if (blockIdx.x == 0) {
      atomicAdd(&J.sc->stats[0], 1ull);
      if (J.sc->fallback) atomicAdd(&J.sc->stats[5], 1ull);
    }
    // the buffer's last decision workgroup to finish closes its latency:
    // wall clock now minus the start its first kernel recorded, against the
    // deadline (the buffer's own real-time span n / fs unless one is set).
    // The count is an atomic and the stamp needs no other workgroup's data,
    // so no fence: a device-scope fence here would write the L2 back once
    // per workgroup (it took the stage from 2.5 to 23 us per buffer).
    const unsigned nwg = (unsigned)((nsym + DEC_SYMS - 1) / DEC_SYMS);
    if (atomicAdd(&J.sc->done_wg, 1u) == nwg - 1) {
      RxScalars *const sc = J.sc;
      const unsigned long long t1 = (unsigned long long)wall_clock64();
      const unsigned long long dt = t1 - *(volatile unsigned long long *)&sc->t_start;
      const double budget = J.deadline_ticks > 0.0 ? J.deadline_ticks : (double)n * J.ticks_per_sample;
      if ((double)dt > budget) atomicAdd(&sc->stats[6], 1ull);
      const unsigned long long c = sc->lat_count;
      sc->lat[c % RX_LAT_RING] = dt < 0xFFFFFFFFull ? (unsigned)dt : 0xFFFFFFFFu;
      sc->lat_count = c + 1;
      sc->done_wg = 0u;
    }
  }
}

// The handle's reference bit stream (Sec. 3: the BER is counted against
// the known transmitted sequence): symbol k is the top bps bits of
// SplitMix64(seed, k), stored like the decided bits (symbol k at stream
// bits [bps k, bps (k + 1)), its most significant bit first).  Filled once
// when the handle is created; every buffer of the handle is compared with it.
__global__ __launch_bounds__(256) void rx_ref_fill(uint32_t *w, int64_t words, uint64_t seed, int bps, int64_t nsym,
                                                   uint64_t period) {
  const int64_t wi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (wi >= words) return;
  uint32_t v = 0u;
  int64_t kc = -1;
  uint32_t sym = 0u;
  for (int b = 0; b < 32; b++) {
    const int64_t sb = 32 * wi + b, k = sb / bps;
    if (k >= nsym) break;
    if (k != kc) {
      kc = k;
      sym = (uint32_t)(splitmix64(seed, period ? (uint64_t)k % period : (uint64_t)k) >> (64 - bps));
    }
    const int j = (int)(sb - k * bps);   // bit j of the field: bit bps - 1 - j of the symbol
    v |= ((sym >> (bps - 1 - j)) & 1u) << b;
  }
  w[wi] = v;
}

void rx_launch_ref_fill(uint32_t *w, int64_t words, uint64_t seed, int bps, int64_t nsym, uint64_t period,
                        hipStream_t s) {
  hipLaunchKernelGGL(rx_ref_fill, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, w, words, seed, bps, nsym,
                     period);
}

void rx_launch_eq_stage(int stage, const RxLaunch &L, int64_t maxn, int kk, int ffe_taps, int prec, const RxTune &t,
                        hipStream_t s) {
  const unsigned cnt = (unsigned)L.count;
  const int64_t nsym = maxn / (kk ? 4 : 2);
  if (stage == ST_PREFIX) {
    hipLaunchKernelGGL(rx_prefix, dim3(1, cnt), dim3(PFX_T), 0, s, L);
  } else if (stage == ST_BLOCKS && kk && prec != 0) {
    const int64_t ngrp = (nsym + 255) / 256;
    const int gpw = t.ffe_gpw;
    dim3 gf((unsigned)((ngrp + 4 * gpw - 1) / (4 * gpw)), cnt);   // four wavefronts per workgroup
#define RX_FFE(P, G) hipLaunchKernelGGL((rx_ffe_mfma<P, G>), gf, dim3(256), 0, s, L)
    if (prec == 1) {
      if (gpw == 4) RX_FFE(1, 4); else if (gpw == 16) RX_FFE(1, 16); else RX_FFE(1, 8);
    } else {
      if (gpw == 4) RX_FFE(2, 4); else if (gpw == 16) RX_FFE(2, 16); else RX_FFE(2, 8);
    }
#undef RX_FFE
  } else if (stage == ST_BLOCKS) {
    const int64_t nb = nsym / (kk ? 128 : 256);
    dim3 gb((unsigned)((nb + 127) / 128), cnt);   // 128 blocks (lane pairs) per workgroup
#define RX_BLK(C, K, B) hipLaunchKernelGGL((rx_blocks<C, K, B>), gb, dim3(256), 0, s, L)
#define RX_BLK_BC(C, K) \
  do { if (t.blocks_bc == 4) RX_BLK(C, K, 4); else if (t.blocks_bc == 16) RX_BLK(C, K, 16); else RX_BLK(C, K, 8); } while (0)
    if (kk) {
      if (ffe_taps == 21) RX_BLK_BC(true, 21);
      else if (ffe_taps == 4) RX_BLK_BC(true, 4);
      else RX_BLK_BC(true, 15);
    } else {
      if (ffe_taps == 21) RX_BLK_BC(false, 21);
      else RX_BLK_BC(false, 15);
    }
#undef RX_BLK_BC
#undef RX_BLK
  } else if (stage == ST_DECIDE) {
    const int ds = t.dec_syms;
    dim3 gd((unsigned)((nsym + ds - 1) / ds), cnt);
    if (ds == 1024) hipLaunchKernelGGL(rx_decide<1024>, gd, dim3(128), 0, s, L);
    else if (ds == 4096) hipLaunchKernelGGL(rx_decide<4096>, gd, dim3(512), 0, s, L);
    else hipLaunchKernelGGL(rx_decide<2048>, gd, dim3(256), 0, s, L);
  }
}

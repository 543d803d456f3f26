// Kramers-Kronig front end for gfx950 (Sec. 2, second paragraph; Fig. 1d).
//
// kk_front: one workgroup per pair of overlap-save blocks.  Two real blocks
// of l = ln(sqrt(v)) share one complex N-point FFT (block A in the real
// part, block B in the imaginary part: the Hilbert filter is real, so the
// two stay separate).  The spectrum is multiplied by the Hilbert response,
// transformed back in LDS, and each sample becomes
//     E = sqrt(v) exp(j phi),  y' = E exp(-j 2 pi frac(r n))
// with the downshift phase accumulated in FP64.  The decimating matched
// filter runs on y' straight from LDS and writes the 2-sample/symbol
// output; only packed codes come in and half-rate complex samples go out.
// The carrier mean m is not known inside one workgroup, so the filter runs
// on y' = y + m exp(-j 2 pi r n); since the filter is linear its consumers
// subtract m * MF(exp(...)) on load, and the AGC power of the carrier-free
// output follows from per-workgroup sums of |Z|^2, |T|^2 and Z conj(T).
#include <type_traits>

#include "fft_lds.hpp"

__device__ __forceinline__ int64_t clamp64(int64_t v, int64_t lo, int64_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Codes of samples s0 .. s0+7 of a frame, replicated beyond the buffer edges.
__device__ __forceinline__ void frame_codes8(const uint8_t *in, int64_t n, int64_t s0, int c[8]) {
  if (s0 >= 0 && s0 + 8 <= n) {
    read_codes8(in, s0 >> 3, c);
  } else {
#pragma unroll
    for (int e = 0; e < 8; e++) c[e] = read_code(in, clamp64(s0 + e, 0, n - 1));
  }
}

__device__ __forceinline__ int ypad(int q) { return q + (q >> 5); }

template <int LOGN, int PREC>
__global__ __launch_bounds__((1 << LOGN) / 16) void kk_front(RxLaunch L) {
  constexpr int N = 1 << LOGN, T = N / 16;
  constexpr int HOP = (N - RX_KK_HALFV - RX_KK_EDGE - RX_KK_CMF) & ~15;
  constexpr int QN = HOP + 2 * RX_KK_CMF;   // y' samples each block needs
  constexpr int QPT = (QN + T - 1) / T;
  constexpr float INV2PI = 0.15915494309189535f;
  __shared__ float2 lds[N + N / 16];
  __shared__ double red[T / 64];
  __shared__ float hev[48], hod[48];   // h[2q], h[2q-1] at index q+8, zero outside the filter

  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const uint8_t *in = L.in[jb];
  const int64_t nrb = (n + HOP - 1) / HOP;
  const int64_t blk[2] = {2 * (int64_t)blockIdx.x, 2 * (int64_t)blockIdx.x + 1};
  if (blk[0] >= nrb) return;
  const int64_t F[2] = {blk[0] * HOP - RX_KK_EDGE, blk[1] * HOP - RX_KK_EDGE};

  if (threadIdx.x < 48) {
    const int q = (int)threadIdx.x - 8;
    hev[threadIdx.x] = (q >= 0 && 2 * q <= 64) ? J.mf[2 * q] : 0.0f;
    hod[threadIdx.x] = (q >= 1 && 2 * q - 1 <= 64) ? J.mf[2 * q - 1] : 0.0f;
  }

  // 1. l - l_ref for both frames (l_ref: the frame's centre sample; the
  //    Hilbert response is zero at DC, so any offset leaves phi unchanged and
  //    a small one keeps the FP32 transform accurate).
  const float off0 = 0.5f * __logf((float)read_code(in, clamp64(F[0] + N / 2, 0, n - 1)) + 0.5f);
  const float off1 = 0.5f * __logf((float)read_code(in, clamp64(F[1] + N / 2, 0, n - 1)) + 0.5f);
  for (int g = threadIdx.x; g < N / 8; g += T) {
    int ca[8], cb[8];
    frame_codes8(in, n, F[0] + 8 * g, ca);
    frame_codes8(in, n, F[1] + 8 * g, cb);
#pragma unroll
    for (int e = 0; e < 8; e++)
      lds[fpad(8 * g + e)] = make_float2(0.5f * __logf((float)ca[e] + 0.5f) - off0,
                                         0.5f * __logf((float)cb[e] + 0.5f) - off1);
  }
  __syncthreads();

  // 2. Hilbert filtering: Y = Z H, H = -j S; the inverse transform is done as
  //    conj(FFT(conj(Y)/N)), so the second pass leaves phiA - j phiB.
  fft_forward<LOGN>(lds, J.twid);
  for (int k = threadIdx.x; k < N; k += T) {
    const float2 zv = lds[fpad(k)];
    const float s = J.hspec[k];
    lds[fpad(k)] = make_float2(zv.y * s, zv.x * s);
  }
  __syncthreads();
  fft_forward<LOGN>(lds, J.twid);

  float ph[2][QPT];
#pragma unroll
  for (int i = 0; i < QPT; i++) {
    const int q = threadIdx.x + i * T;
    if (q < QN) {
      const float2 v = lds[fpad(q + RX_KK_EDGE - RX_KK_CMF)];
      ph[0][i] = v.x * J.sgn * INV2PI;
      ph[1][i] = -v.y * J.sgn * INV2PI;
    }
  }
  __syncthreads();

  double se_re = 0.0, se_im = 0.0;
  double zz = 0.0, tt = 0.0, ztr = 0.0, zti = 0.0;   // sum |Z|^2, |T|^2, Z conj(T)
  auto zstat = [&](int64_t m, float2 zv, float2 tc) {
    zz += (double)zv.x * zv.x + (double)zv.y * zv.y;
    tt += (double)tc.x * tc.x + (double)tc.y * tc.y;
    const float2 p = cmulc(zv, tc);
    ztr += p.x;
    zti += p.y;
  };
#pragma unroll
  for (int x = 0; x < 2; x++) {
    // 3. field, carrier mean partials, downshifted field y' into LDS
    const int64_t nq0 = F[x] + RX_KK_EDGE - RX_KK_CMF;   // sample index of q = 0
#pragma unroll
    for (int i = 0; i < QPT; i++) {
      const int q = threadIdx.x + i * T;
      if (q < QN) {
        const int64_t t = nq0 + q;
        float2 yv = make_float2(0.0f, 0.0f);
        if (t >= 0 && t < n) {
          const float mag = sqrtf((float)read_code(in, t) + 0.5f);
          const float u = downshift_rev(J.r, t);
          yv = cscale(cis_rev(ph[x][i] - u), mag);
          if (q >= RX_KK_CMF && q < RX_KK_CMF + HOP) {
            const float2 e = cscale(cis_rev(ph[x][i]), mag);
            se_re += e.x;
            se_im += e.y;
            if (J.field) J.field[t] = e;
          }
        }
        lds[ypad(q)] = yv;
      }
    }
    __syncthreads();
    const int64_t m0 = blk[x] * (HOP / 2);
    if constexpr (PREC == 0) {
      // 4. decimating matched filter Z[m] = sum_i h[i] y'[2m + 32 - i], eight
      //    consecutive outputs per thread.  Polyphase form: at step e the input
      //    pair y'(2e), y'(2e+1) meets the even taps h[2(o+32-e)] and the odd
      //    taps h[2(o+32-e)-1] of outputs o = 0..7; those taps form an 8-wide
      //    window that slides by one per step, so each step loads one even and
      //    one odd tap (zero-padded tables in LDS) and two inputs.
      for (int t8 = threadIdx.x; t8 < HOP / 16; t8 += T) {
        float2 acc[8];
        float we[8], wo[8];
  #pragma unroll
        for (int o = 0; o < 8; o++) {
          acc[o] = make_float2(0.0f, 0.0f);
          we[o] = hev[32 + o + 8];
          wo[o] = hod[32 + o + 8];
        }
        const int qb = 16 * t8;
  #pragma unroll 1
        for (int eb = 0; eb < 40; eb += 8) {
  #pragma unroll
          for (int ee = 0; ee < 8; ee++) {
            const int e = eb + ee;
            const float2 y0 = lds[ypad(qb + 2 * e)];
            const float2 y1 = lds[ypad(qb + 2 * e + 1)];
  #pragma unroll
            for (int o = 0; o < 8; o++) {
              const int slot = (o - ee + 8) & 7;
              acc[o].x = fmaf(we[slot], y0.x, acc[o].x);
              acc[o].y = fmaf(we[slot], y0.y, acc[o].y);
              acc[o].x = fmaf(wo[slot], y1.x, acc[o].x);
              acc[o].y = fmaf(wo[slot], y1.y, acc[o].y);
            }
            // next step's window: slot (-e-1) mod 8 takes h(31 - e)
            we[(7 - ee) & 7] = hev[31 - e + 8];
            wo[(7 - ee) & 7] = hod[31 - e + 8];
          }
        }
        // carrier term of the 8 outputs: exact at the first, then rotated by
        // exp(-j 4 pi r) (it enters only the AGC power sums)
        const int64_t mb = m0 + 8 * t8;
        float2 tc = kk_carrier_term(J, mb, n);
#pragma unroll
        for (int o = 0; o < 8; o++) {
          const int64_t m = mb + o;
          if (2 * m < n) {
            J.z[m] = acc[o];
            if (o > 0) tc = kk_interior(m, n) ? cmul(tc, J.rot2) : kk_carrier_term(J, m, n);
            zstat(m, acc[o], tc);
          }
        }
      }

    } else {
      // 4'. precision form: the same filter as a Toeplitz GEMM on MFMA with
      //     narrow operands and FP32 accumulation.  A row = one real
      //     component (re or im) of the 96-sample window of a tile of 16
      //     outputs, B[t][q] = h[2q + 64 - t]; one 16x16x32 step per 32
      //     window samples, eight tiles (16 rows) per wavefront pass.
      using NT = NarrowT<PREC>;
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      constexpr int NTILE = HOP / 32;
      const int row = lane & 15, kq = lane >> 4;
      typename NT::vec bmf[3];   // B fragments of the tap matrix
#pragma unroll
      for (int ks = 0; ks < 3; ks++)
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const int t = 32 * ks + 8 * kq + j, tap = 2 * row + 64 - t;
          bmf[ks][j] = NT::cvt((tap >= 0 && tap <= 64) ? J.mf[tap] : 0.0f);
        }
      for (int grp = wv; grp < (NTILE + 7) / 8; grp += T / 64) {
        const int tile = grp * 8 + (row >> 1);
        rx_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 3; ks++) {
          typename NT::vec a;
#pragma unroll
          for (int j = 0; j < 8; j++) {
            const float2 v = lds[ypad(32 * tile + 32 * ks + 8 * kq + j)];
            a[j] = NT::cvt((row & 1) ? v.y : v.x);
          }
          acc = NT::mfma(a, bmf[ks], acc);
        }
#pragma unroll
        for (int jj = 0; jj < 2; jj++) {
          const int t2 = grp * 8 + 2 * kq + jj;
          const int64_t m = m0 + 16 * t2 + row;
          if (t2 < NTILE && 2 * m < n) {
            const float2 zv = make_float2(acc[2 * jj], acc[2 * jj + 1]);
            J.z[m] = zv;
            zstat(m, zv, kk_carrier_term(J, m, n));
          }
        }
      }
    }
    __syncthreads();
  }
  const double sr = block_sum(se_re, red), si = block_sum(se_im, red);
  const double szz = block_sum(zz, red), stt = block_sum(tt, red);
  const double szr = block_sum(ztr, red), szi = block_sum(zti, red);
  if (threadIdx.x == 0) {
    J.part[3 * blockIdx.x] = make_double2(sr, si);          // sum of the field E
    J.part[3 * blockIdx.x + 1] = make_double2(szz, stt);    // sum |Z|^2, sum |T|^2
    J.part[3 * blockIdx.x + 2] = make_double2(szr, szi);    // sum Z conj(T)
  }
}

// Debug only (RX_DEBUG_KEEP): materialise u[m] = g (Z[m] - mean T[m]) exactly
// as the consumers form it on load.
__global__ __launch_bounds__(256) void kk_debug_u(RxLaunch L) {
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  if (!J.udbg) return;
  const int64_t n = L.n[jb];
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= n / 2) return;
  const float2 mean = make_float2((float)J.sc->mean_re, (float)J.sc->mean_im);
  J.udbg[m] = kk_sample(J, J.z, m, n, mean, (float)J.sc->agc);
}

// Viterbi-Viterbi carrier phase per DD-LMS block over blocks b-1..b+1,
// unwrapped in multiples of pi/2 (wrapped differences, then a workgroup
// prefix sum), one workgroup per buffer.
__global__ __launch_bounds__(1024) void kk_vv(RxLaunch L) {
  __shared__ double scan[1024];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t nsym = L.n[jb] / 4;
  const int nb = (int)(nsym / J.blk);
  const int per = (nb + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  constexpr float Q = 1.5707963267948966f;
  auto raw = [&](int b) {
    float2 s = J.s4[b];
    if (b > 0) s = cadd(s, J.s4[b - 1]);
    if (b + 1 < nb) s = cadd(s, J.s4[b + 1]);
    return 0.25f * atan2f(-s.y, -s.x);
  };
  auto wrapq = [&](float d) { return d - Q * floorf(d / Q + 0.5f); };
  double local = 0.0;
  float prev = (b0 > 0 && b0 < nb) ? raw(b0 - 1) : 0.0f;
  for (int b = b0; b < b0 + per && b < nb; b++) {
    const float r = raw(b);
    local += (b == 0) ? r : wrapq(r - prev);
    prev = r;
  }
  scan[threadIdx.x] = local;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const double v = threadIdx.x >= o ? scan[threadIdx.x - o] : 0.0;
    __syncthreads();
    scan[threadIdx.x] += v;
    __syncthreads();
  }
  double th = scan[threadIdx.x] - local;   // exclusive prefix
  prev = (b0 > 0 && b0 < nb) ? raw(b0 - 1) : 0.0f;
  for (int b = b0; b < b0 + per && b < nb; b++) {
    const float r = raw(b);
    th += (b == 0) ? r : wrapq(r - prev);
    prev = r;
    J.theta[b] = (float)th;
  }
}

template <int LOGN, int PREC>
static void launch_front(const RxLaunch &L, int64_t maxn, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  const int hop = rx_kk_hop(LOGN);
  const int64_t nrb = (maxn + hop - 1) / hop;
  dim3 grid((unsigned)((nrb + 1) / 2), (unsigned)L.count);
  hipLaunchKernelGGL((kk_front<LOGN, PREC>), grid, dim3(N / 16), 0, s, L);
}

void rx_launch_kk_stage(int stage, const RxLaunch &L, int64_t maxn, int log2n, int prec, hipStream_t s) {
  const unsigned cnt = (unsigned)L.count;
  if (stage == ST_KK_FRONT) {
    if (log2n == 13) {
      if (prec == 1) launch_front<13, 1>(L, maxn, s);
      else if (prec == 2) launch_front<13, 2>(L, maxn, s);
      else launch_front<13, 0>(L, maxn, s);
    } else {
      if (prec == 1) launch_front<14, 1>(L, maxn, s);
      else if (prec == 2) launch_front<14, 2>(L, maxn, s);
      else launch_front<14, 0>(L, maxn, s);
    }
  } else if (stage == ST_KK_DEBUG) {
    const int64_t nd = maxn / 2;
    hipLaunchKernelGGL(kk_debug_u, dim3((unsigned)((nd + 255) / 256), cnt), dim3(256), 0, s, L);
  } else if (stage == ST_KK_VV) {
    hipLaunchKernelGGL(kk_vv, dim3(1, cnt), dim3(1024), 0, s, L);
  }
}

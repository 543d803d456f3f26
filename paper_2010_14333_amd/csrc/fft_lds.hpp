// In-LDS complex FFT for one workgroup: Stockham auto-sort, radix-16 passes
// followed by one radix-2/4/8 pass, N = 16 * blockDim.x (or radix-8 passes,
// N = 8 * blockDim.x).  Each thread holds exactly 16 (8) values per pass:
// read all, barrier, butterfly, write, barrier, so the transform runs in
// place in one padded LDS buffer.  The passes can
// be entered after the first (a caller that formed the first pass itself)
// and the last pass's outputs handed to a caller's functor instead of LDS.
#pragma once
#include "rx_dev.hpp"

// threadIdx.x as a value the compiler cannot treat as loop-invariant: in a
// kernel that loops over work items, the per-thread addresses of each pass
// are then formed inside the iteration instead of being hoisted out of the
// loop and held in registers (or scratch) across all of it.
__device__ __forceinline__ int tid_local() {
  unsigned t = threadIdx.x;
  asm volatile("" : "+v"(t));
  __builtin_assume(t < 1024u);   // the range the compiler knew of threadIdx.x
  return (int)t;
}

// Orders one wavefront's LDS accesses across lanes: its DS instructions
// execute in program order, so a fence that keeps the compiler from moving
// accesses across it is all that a wavefront-local exchange needs.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS index with one float2 of padding every 16: stride-16 writes of the
// first pass then spread over all banks.
__host__ __device__ constexpr int fpad(int p) { return p + (p >> 4); }

__device__ __forceinline__ float2 mul_mj(float2 a) { return make_float2(a.y, -a.x); }  // -j * a

__device__ __forceinline__ void dft2(float2 &a, float2 &b) {
  const float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

// 4-point forward DFT (kernel exp(-j 2 pi kn/4)), natural order in and out.
__device__ __forceinline__ void dft4(float2 &x0, float2 &x1, float2 &x2, float2 &x3) {
  const float2 t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3), t3 = mul_mj(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

// 8-point forward DFT as 2 x 4 (natural order in and out).
__device__ __forceinline__ void dft8(float2 *v) {
  const float h = 0.70710678118654752f;
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  o1 = make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));   // * exp(-j pi/4)
  o2 = mul_mj(o2);                                          // * exp(-j pi/2)
  o3 = make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));  // * exp(-j 3pi/4)
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// 16-point forward DFT as 4 x 4: X[k1 + 4 k2] = sum_n2 W16^(n2 k1) W4^(n2 k2)
// sum_n1 x[4 n1 + n2] W4^(n1 k1).  The inner 4-point DFTs give p_n2 (for
// each k1); column k1 then takes q_n = W16^(n k1) p_n through a 4-point
// DFT.  Each rotation is written as a real scale times a vector with one
// FMA per component (W^1 p = c (p.x + t p.y, p.y - t p.x), W^3 p =
// c (t p.x + p.y, t p.y - p.x), c = cos(pi/8), t = tan(pi/8); W^2 and W^6 p
// = h times sums, h = sqrt(1/2); W^9 = -W^1), and the scale rides in the
// FMAs of the column's butterflies: 144 instructions instead of 160.
__device__ __forceinline__ void dft16(float2 *v) {
  const float c1 = 0.92387953251128674f, tn = 0.41421356237309505f, h = 0.70710678118654752f;
  float2 a[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; n2++) {
    float2 x0 = v[n2], x1 = v[4 + n2], x2 = v[8 + n2], x3 = v[12 + n2];
    dft4(x0, x1, x2, x3);
    a[n2 * 4 + 0] = x0; a[n2 * 4 + 1] = x1; a[n2 * 4 + 2] = x2; a[n2 * 4 + 3] = x3;
  }
  // column k1 = 0: no rotations
  {
    float2 x0 = a[0], x1 = a[4], x2 = a[8], x3 = a[12];
    dft4(x0, x1, x2, x3);
    v[0] = x0; v[4] = x1; v[8] = x2; v[12] = x3;
  }
  // X0 = u0 + f s, X2 = u0 - f s, X1 = u1 - j f d, X3 = u1 + j f d
  auto close = [](float2 u0, float2 u1, float2 s, float2 d, float f, float2 &x0, float2 &x1, float2 &x2, float2 &x3) {
    x0 = make_float2(fmaf(f, s.x, u0.x), fmaf(f, s.y, u0.y));
    x2 = make_float2(fmaf(-f, s.x, u0.x), fmaf(-f, s.y, u0.y));
    x1 = make_float2(fmaf(f, d.y, u1.x), fmaf(-f, d.x, u1.y));
    x3 = make_float2(fmaf(-f, d.y, u1.x), fmaf(f, d.x, u1.y));
  };
  // column k1 = 1: q1 = c b1, q2 = h b2, q3 = c b3
  {
    const float2 p0 = a[1], p1 = a[5], p2 = a[9], p3 = a[13];
    const float2 b1 = make_float2(fmaf(tn, p1.y, p1.x), fmaf(-tn, p1.x, p1.y));
    const float2 b3 = make_float2(fmaf(tn, p3.x, p3.y), fmaf(tn, p3.y, -p3.x));
    const float2 b2 = make_float2(p2.x + p2.y, p2.y - p2.x);
    const float2 u0 = make_float2(fmaf(h, b2.x, p0.x), fmaf(h, b2.y, p0.y));
    const float2 u1 = make_float2(fmaf(-h, b2.x, p0.x), fmaf(-h, b2.y, p0.y));
    close(u0, u1, cadd(b1, b3), csub(b1, b3), c1, v[1], v[5], v[9], v[13]);
  }
  // column k1 = 2: q1 = h b1, q2 = -j p2, q3 = h b3
  {
    const float2 p0 = a[2], p1 = a[6], p2 = a[10], p3 = a[14];
    const float2 b1 = make_float2(p1.x + p1.y, p1.y - p1.x);
    const float2 b3 = make_float2(p3.y - p3.x, -p3.x - p3.y);
    const float2 u0 = make_float2(p0.x + p2.y, p0.y - p2.x);
    const float2 u1 = make_float2(p0.x - p2.y, p0.y + p2.x);
    close(u0, u1, cadd(b1, b3), csub(b1, b3), h, v[2], v[6], v[10], v[14]);
  }
  // column k1 = 3: q1 = c b1, q2 = h b2, q3 = -c b3
  {
    const float2 p0 = a[3], p1 = a[7], p2 = a[11], p3 = a[15];
    const float2 b1 = make_float2(fmaf(tn, p1.x, p1.y), fmaf(tn, p1.y, -p1.x));
    const float2 b3 = make_float2(fmaf(tn, p3.y, p3.x), fmaf(-tn, p3.x, p3.y));
    const float2 b2 = make_float2(p2.y - p2.x, -p2.x - p2.y);
    const float2 u0 = make_float2(fmaf(h, b2.x, p0.x), fmaf(h, b2.y, p0.y));
    const float2 u1 = make_float2(fmaf(-h, b2.x, p0.x), fmaf(-h, b2.y, p0.y));
    close(u0, u1, csub(b1, b3), cadd(b1, b3), c1, v[3], v[7], v[11], v[15]);
  }
}

template <int R>
__device__ __forceinline__ void dft_r(float2 *v) {
  if constexpr (R == 16) dft16(v);
  else if constexpr (R == 8) dft8(v);
  else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
  else dft2(v[0], v[1]);
}

// Twiddle W^r (r < 16) from the table powers W, W^2, W^4, W^8: at most three
// products deep, so the error stays a few ulp.
template <int r>
__device__ __forceinline__ float2 twid_pow(float2 w1, float2 w2, float2 w4, float2 w8) {
  float2 w = make_float2(1.0f, 0.0f);
  bool first = true;
  if constexpr ((r & 1) != 0) { w = w1; first = false; }
  if constexpr ((r & 2) != 0) { w = first ? w2 : cmul(w, w2); first = false; }
  if constexpr ((r & 4) != 0) { w = first ? w4 : cmul(w, w4); first = false; }
  if constexpr ((r & 8) != 0) { w = first ? w8 : cmul(w, w8); }
  return w;
}

template <int R, int I>
__device__ __forceinline__ void apply_twiddles(float2 *v, float2 w1, float2 w2, float2 w4, float2 w8) {
  if constexpr (I < R) {
    v[I] = cmul(v[I], twid_pow<I>(w1, w2, w4, w8));
    apply_twiddles<R, I + 1>(v, w1, w2, w4, w8);
  }
}

// Where a pass puts its outputs.  begin() runs at the start of the pass,
// before its LDS reads (a place to issue loads the outputs will need);
// out(koff, pk, v) takes output v, with koff = its index minus threadIdx.x
// (a constant once the loops are unrolled; meaningful in the last pass,
// whose butterfly j = threadIdx.x + b T writes outputs j + r NS) and pk its
// padded LDS slot.  The default writes the slot; a caller can take the last
// pass's outputs in registers instead.
struct LdsOut {
  float2 *buf;
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ void operator()(int, int pk, float2 v) const { buf[pk] = v; }
};

// One Stockham pass of radix R with NS = product of the previous radices.
// Butterfly j reads x[j + r N/R], twiddles by W_{NS R}^{r (j mod NS)}, and
// writes to (j / NS) NS R + (j mod NS) + r NS.  NS is a compile-time
// constant so the padded LDS offsets of the VPT accesses fold to immediates.
// TWL: every twiddle W^r read from the table (R - 1 loads a butterfly and no
// products), else W, W^2, W^4, W^8 read and the others formed as their
// products.  With the table in natural order the R - 1 loads of a wavefront
// touch about four times the cache lines of the four (lane stride 8 r NS'
// bytes), which costs the 2^14-point front end far more than the products
// it saves; it stays off there.
// WV: a transform of one wavefront (T = 64 lanes, buf its own LDS region),
// synchronised by wave_sync instead of workgroup barriers.
template <int N, int R, int NS, bool TAIL = true, class Out = LdsOut, int VPT = 16, bool TWL = false,
          bool WV = false>
__device__ __forceinline__ void stockham_pass(float2 *buf, const float2 *__restrict__ tw, Out out) {
  constexpr int T = N / VPT;
  constexpr int NB = (N / R) / T;  // butterflies per thread
  static_assert(!WV || T == 64, "a wavefront transform has one butterfly column per lane");
  const int tx = WV ? (tid_local() & 63) : tid_local();
  // twiddle table reads first: their latency overlaps the LDS reads and the
  // barrier.  They go through a global-memory view: as flat accesses they
  // would also count against the LDS wait counter, and the wait for this
  // pass's LDS reads would wait for them too.
  float2 tw1[NB], tw2[NB], tw4[NB], tw8[NB];
  float2 twr[TWL ? NB : 1][TWL ? R : 1];
  if constexpr (NS > 1) {
    const GView2 tg = gview(tw);
#pragma unroll
    for (int b = 0; b < NB; b++) {
      const int j = tx + b * T;
      const unsigned step = (unsigned)(j & (NS - 1)) * (N / (NS * R));   // r step < N
      if constexpr (TWL) {
#pragma unroll
        for (int r = 1; r < R; r++) twr[b][r] = tg.at(r * step);
      } else {
        tw1[b] = tg.at(step);
        tw2[b] = R > 2 ? tg.at(2 * step) : tw1[b];
        tw4[b] = R > 4 ? tg.at(4 * step) : tw1[b];
        tw8[b] = R > 8 ? tg.at(8 * step) : tw1[b];
      }
    }
  }
  out.begin();
  float2 v[NB][R];
  // N / R is a multiple of 16, so fpad(j + r N/R) = fpad(j) + fpad(r N/R):
  // one address per butterfly, the rest immediate offsets
  static_assert((N / R) % 16 == 0, "padded read offsets split");
  // (the reads past 64 KiB of the first take a second base: the offset
  // field of an LDS read holds 16 bits)
  constexpr bool TWO = 8 * fpad((R - 1) * (N / R)) >= 65536;
  constexpr int RH = TWO ? R / 2 : R, OH = fpad(RH * (N / R));
#pragma unroll
  for (int b = 0; b < NB; b++) {
    const int pj = fpad(tx + b * T);
    int pj1 = pj + OH;
    if constexpr (TWO) asm volatile("" : "+v"(pj1));   // kept as its own base, not refolded into pj
    const float2 *b0 = buf + pj, *b1 = buf + pj1;
#pragma unroll
    for (int r = 0; r < R; r++) v[b][r] = r < RH ? b0[fpad(r * (N / R))] : b1[fpad(r * (N / R)) - OH];
  }
  // in the last pass (NS R = N) a butterfly writes back exactly the indices
  // it read, so no thread overwrites another's input: no barrier needed
  if constexpr (NS * R != N) {
    if constexpr (WV) wave_sync();
    else __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < NB; b++) {
    const int j = tx + b * T;
    const int k = j & (NS - 1);
    if constexpr (NS > 1 && TWL) {
#pragma unroll
      for (int r = 1; r < R; r++) v[b][r] = cmul(v[b][r], twr[b][r]);
    } else if constexpr (NS > 1) {
      apply_twiddles<R, 1>(v[b], tw1[b], tw2[b], tw4[b], tw8[b]);
    }
    dft_r<R>(v[b]);
    const int base = (j / NS) * NS * R + k;
    // fpad(base + r NS) = fpad(base) + fpad(r NS): either NS is a multiple of
    // 16, or base mod 16 + r NS mod 16 < 16 (NS = 1, R = 16: base mod 16 = 0;
    // NS = 1 or 8, R = 8: base mod 16 < 8 and r NS mod 16 in {0, 8} or < 8);
    // the second term is a constant, folded into the store's offset
    static_assert(NS % 16 == 0 || (NS == 1 && (R == 16 || R == 8)) || (NS == 8 && R == 8),
                  "padded write offsets split");
    const int pb = fpad(base);
#pragma unroll
    for (int r = 0; r < R; r++) out(b * T + r * NS, pb + fpad(r * NS), v[b][r]);
  }
  if constexpr (TAIL) {
    if constexpr (WV) wave_sync();
    else __syncthreads();
  }
}

// Radix-8 passes only, 8 values per thread (N = 8 * blockDim.x, N a power of 8).
template <int N, int NS, bool TAIL, class Out>
__device__ __forceinline__ void fft_passes8(float2 *buf, const float2 *__restrict__ tw, Out out) {
  if constexpr (NS * 8 < N) {
    stockham_pass<N, 8, NS, true, LdsOut, 8>(buf, tw, LdsOut{buf});
    fft_passes8<N, NS * 8, TAIL>(buf, tw, out);
  } else {
    static_assert(NS * 8 == N, "N is a power of 8");
    stockham_pass<N, 8, NS, TAIL, Out, 8>(buf, tw, out);
  }
}

template <int N, int NS, bool TAIL, class Out, bool TWL = false, bool WV = false>
__device__ __forceinline__ void fft_passes(float2 *buf, const float2 *__restrict__ tw, Out out) {
  if constexpr (NS * 16 < N) {
    stockham_pass<N, 16, NS, true, LdsOut, 16, TWL, WV>(buf, tw, LdsOut{buf});
    fft_passes<N, NS * 16, TAIL, Out, TWL, WV>(buf, tw, out);
  } else if constexpr (NS * 16 == N) {
    stockham_pass<N, 16, NS, TAIL, Out, 16, TWL, WV>(buf, tw, out);
  } else if constexpr (NS * 8 == N) {
    stockham_pass<N, 8, NS, TAIL, Out, 16, TWL, WV>(buf, tw, out);
  } else if constexpr (NS * 4 == N) {
    stockham_pass<N, 4, NS, TAIL, Out, 16, TWL, WV>(buf, tw, out);
  } else if constexpr (NS * 2 == N) {
    stockham_pass<N, 2, NS, TAIL, Out, 16, TWL, WV>(buf, tw, out);
  }
}

// Forward FFT of N = 2^LOGN points held in buf (padded layout), natural
// order in.  tw[k] = exp(-j 2 pi k / N).  Output k comes from thread
// k mod (N / 16) and goes to out (default: natural order in buf); with
// TAIL = false the last pass ends without a barrier, for a caller whose
// threads next touch only their own outputs.
template <int LOGN, bool TAIL = true, class Out = LdsOut>
__device__ __forceinline__ void fft_forward(float2 *buf, const float2 *__restrict__ tw, Out out) {
  fft_passes<(1 << LOGN), 1, TAIL>(buf, tw, out);
}
template <int LOGN, bool TAIL = true>
__device__ __forceinline__ void fft_forward(float2 *buf, const float2 *__restrict__ tw) {
  fft_passes<(1 << LOGN), 1, TAIL>(buf, tw, LdsOut{buf});
}

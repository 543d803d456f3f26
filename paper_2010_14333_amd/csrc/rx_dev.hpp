// Device helpers for the gfx950 receiver kernels (wave64).
#pragma once
#include "rx_shared.h"

#define RX_WAVE 64

typedef __bf16 rx_bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 rx_f16x8 __attribute__((ext_vector_type(8)));
typedef float rx_f32x4 __attribute__((ext_vector_type(4)));
typedef float rx_f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 rx_f16x2 __attribute__((ext_vector_type(2)));

// Narrow operand type of the precision form (PREC 1: BF16, 2: FP16), with
// round-to-nearest-even conversion from FP32.
template <int PREC> struct NarrowT;
template <> struct NarrowT<1> {
  using vec = rx_bf16x8;
  using elem = __bf16;
  __device__ static __bf16 cvt(float v) { return (__bf16)v; }
  __device__ static rx_f32x4 mfma(vec a, vec b, rx_f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct NarrowT<2> {
  using vec = rx_f16x8;
  using elem = _Float16;
  __device__ static _Float16 cvt(float v) { return (_Float16)v; }
  __device__ static rx_f32x4 mfma(vec a, vec b, rx_f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
// Operand layout of v_mfma_f32_16x16x32_{bf16,f16}: lane l supplies
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16], j = 0..7, and
// receives D[4 (l / 16) + j][l % 16], j = 0..3.

// Global-memory view of a pointer.  Pointers read out of the job descriptor
// are generic to the compiler, which then emits flat accesses; those also
// count against the LDS wait counter, so every wait for an LDS read would
// wait for outstanding HBM loads too.  Hot paths access through this view.
// (HIP's float2/float4 classes do not bind to address-space-qualified
// references, so complex and 4-wide accesses go through native vectors.)
#define RX_GLOBAL __attribute__((address_space(1)))
typedef float rx_v2 __attribute__((ext_vector_type(2)));
typedef float rx_v4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ RX_GLOBAL T *gptr(T *p) { return (RX_GLOBAL T *)p; }
// Element i (i < 2^32 / sizeof(T)) of a global array with a uniform base:
// a 32-bit unsigned byte offset lets the load take the base in scalar
// registers and one vector register of offset, with no 64-bit address
// arithmetic per thread.
template <class T>
__device__ __forceinline__ T gload_u32(const T *base, unsigned i) {
  return *(const RX_GLOBAL T *)((const RX_GLOBAL char *)base + i * (unsigned)sizeof(T));
}
struct GView2 {   // read-only global view of a float2 array
  const RX_GLOBAL rx_v2 *p;
  __device__ float2 operator[](int64_t i) const {
    const rx_v2 v = p[i];
    return make_float2(v.x, v.y);
  }
  __device__ float2 at(unsigned i) const {   // i < 2^29, as gload_u32
    const rx_v2 v = *(const RX_GLOBAL rx_v2 *)((const RX_GLOBAL char *)p + i * 8u);
    return make_float2(v.x, v.y);
  }
};
__device__ __forceinline__ GView2 gview(const float2 *p) { return GView2{(const RX_GLOBAL rx_v2 *)p}; }
__device__ __forceinline__ void gstore(float2 *p, int64_t i, float2 v) {
  ((RX_GLOBAL rx_v2 *)p)[i] = rx_v2{v.x, v.y};
}
__device__ __forceinline__ void gstore_u32(float2 *p, unsigned i, float2 v) {   // i < 2^29, as gload_u32
  *(RX_GLOBAL rx_v2 *)((RX_GLOBAL char *)p + i * 8u) = rx_v2{v.x, v.y};
}
__device__ __forceinline__ float4 gload4(const void *p, int64_t i) {   // i-th 16-byte element
  const rx_v4 v = ((const RX_GLOBAL rx_v4 *)p)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// ---- wave / workgroup reductions ---------------------------------------
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, RX_WAVE);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, RX_WAVE);
  return v;
}
// A double from another lane of the same row of 16, by DPP: each 32-bit
// half moves as a VALU operand, without the LDS crossbar of a shuffle.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// Sum of a double over the wavefront, every lane getting it: within each row
// of 16 lanes by DPP (partners lane ^ 1, lane ^ 2 (quad permutes), then the
// half-row and row mirrors, which pair the two sums formed so far), across
// rows by two shuffles.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  v += dpp_f64<0x140>(v);   // row_mirror
  v += __shfl_xor(v, 16, RX_WAVE);
  v += __shfl_xor(v, 32, RX_WAVE);
  return v;
}
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, RX_WAVE);
  return v;
}

// Sum of a double over the workgroup; every thread gets the result.
// `scratch` holds at least blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double *scratch) {
  v = wave_sum(v);
  const int w = threadIdx.x / RX_WAVE, nw = blockDim.x / RX_WAVE;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; i++) s += scratch[i];
  __syncthreads();
  return s;
}

// Sums of K doubles over the workgroup, in place (every thread gets them).
// `scratch` holds at least K * blockDim.x / 64 doubles.
template <int K>
__device__ __forceinline__ void block_sum_n(double *v, double *scratch) {
  const int w = threadIdx.x / RX_WAVE, nw = blockDim.x / RX_WAVE;
#pragma unroll
  for (int k = 0; k < K; k++) v[k] = wave_sum(v[k]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < K; k++) scratch[k * nw + w] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; k++) {
    double s = 0.0;
    for (int i = 0; i < nw; i++) s += scratch[k * nw + i];
    v[k] = s;
  }
  __syncthreads();
}

// ---- reference sequence (SplitMix64, Steele, Lea & Flood 2014) -----------
#define RX_SM64_GAMMA 0x9E3779B97F4A7C15ull
// SplitMix64 output mixing of the state z = seed + (k + 1) gamma
__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  return splitmix64_mix(seed + (k + 1ull) * RX_SM64_GAMMA);
}

__device__ __forceinline__ uint32_t gray_inverse(uint32_t g) {
  uint32_t i = g;
  for (uint32_t s = g >> 1; s; s >>= 1) i ^= s;
  return i;
}

// Bits of symbol k in a reference stream packed like the output (symbol k
// at stream bits [bps k, bps (k + 1)), its most significant bit first).
__device__ __forceinline__ uint32_t ref_stream_bits(const RxJob &J, int64_t k) {
  const int64_t ob = (int64_t)J.bps * k;
  uint64_t v = J.refw[ob >> 5];
  if ((ob & 31) + J.bps > 32) v |= (uint64_t)J.refw[(ob >> 5) + 1] << 32;
  const uint32_t f = (uint32_t)(v >> (ob & 31)) & ((1u << J.bps) - 1u);
  return __builtin_bitreverse32(f) >> (32 - J.bps);
}

// Bits of symbol k of the seeded reference sequence (top bps bits of the
// k-th SplitMix64 output; the sequence repeats every ref_period symbols when
// that is set, as a transmitter repeating a finite pattern does).
__device__ __forceinline__ uint32_t ref_seed_bits(const RxJob &J, int64_t k) {
  const uint64_t kr = J.ref_period ? (uint64_t)k % J.ref_period : (uint64_t)k;
  return (uint32_t)(splitmix64(J.seed, kr) >> (64 - J.bps));
}

// Transmitted symbol k (stream index) in odd-integer units (QAM: I bits
// first): from the caller's reference stream if the handle has one, else
// from the seed.
__device__ __forceinline__ float2 ref_symbol(const RxJob &J, int64_t k) {
  const uint32_t b = J.ref_ext ? ref_stream_bits(J, k) : ref_seed_bits(J, k);
  const int m = J.m_axis;
  if (J.kk) {
    const int half = J.bps >> 1;
    const uint32_t bi = b >> half, bq = b & (uint32_t)(m - 1);
    return make_float2((float)(2 * (int)gray_inverse(bi) - (m - 1)),
                       (float)(2 * (int)gray_inverse(bq) - (m - 1)));
  }
  return make_float2((float)(2 * (int)gray_inverse(b) - (m - 1)), 0.0f);
}

// ---- decisions: levels 2i-(M-1), thresholds at even integers, tie -> up ---
// floor((v + m) / 2) is computed as floor(fma(v, 1/2, m/2)): scaling by 1/2
// is exact, so both round v + m once.  The clamp uses v_med3 directly (no
// NaN canonicalisation of the operands).
__device__ __forceinline__ float decide_floor(float v, int m) {
  const float f = floorf(fmaf(v, 0.5f, 0.5f * (float)m));
  return __builtin_amdgcn_fmed3f(f, 0.0f, (float)(m - 1));
}
__device__ __forceinline__ int decide_index(float v, int m) { return (int)decide_floor(v, m); }
__device__ __forceinline__ float decide_level(float v, int m) {
  return fmaf(2.0f, decide_floor(v, m), (float)(1 - m));
}

// ---- 12-bit packed input -------------------------------------------------
// Code of sample i (any i in range): the 16 bits at byte 3i/2 hold it in
// their low 12 bits (even i) or high 12 bits (odd i).
__device__ __forceinline__ int read_code(const uint8_t *in, int64_t i) {
  const uint8_t *b = in + ((3 * i) >> 1);
  const int v = (int)b[0] | ((int)b[1] << 8);
  return (v >> ((int)(i & 1) << 2)) & 0xFFF;
}

// Eight codes of samples 8g .. 8g+7 from the three aligned 32-bit words
// that hold them.
__device__ __forceinline__ void unpack_codes8(uint32_t w0, uint32_t w1, uint32_t w2, int c[8]) {
  c[0] = w0 & 0xFFF;
  c[1] = (w0 >> 12) & 0xFFF;
  c[2] = (w0 >> 24) | ((w1 & 0xF) << 8);
  c[3] = (w1 >> 4) & 0xFFF;
  c[4] = (w1 >> 16) & 0xFFF;
  c[5] = (w1 >> 28) | ((w2 & 0xFF) << 4);
  c[6] = (w2 >> 8) & 0xFFF;
  c[7] = w2 >> 20;
}
__device__ __forceinline__ void read_codes8(const uint8_t *in, int64_t g, int c[8]) {
  const uint32_t *p = reinterpret_cast<const uint32_t *>(in + 12 * g);
  unpack_codes8(p[0], p[1], p[2], c);
}

// exp(-j 2 pi frac(r n)) with the phase accumulator in FP64.
__device__ __forceinline__ float downshift_rev(double r, int64_t n) {
  double u = r * (double)n;
  u -= floor(u);
  return (float)u;
}
// exp(+j 2 pi rev) from the hardware sine/cosine, whose argument is in
// revolutions (valid for |rev| < 256).
__device__ __forceinline__ float2 cis_rev(float rev) {
  return make_float2(__builtin_amdgcn_cosf(rev), __builtin_amdgcn_sinf(rev));
}

// KK: the matched filter's response to the downshifted carrier,
// T[m] = sum_i h[i] exp(-j 2 pi frac(r (g0 + 2m + 32 - i))) over in-range samples
// (g0: stream index of the input's first sample, 0 for an independent buffer);
// in the interior it is c0 exp(-j 2 pi frac(r (g0 + 2m))).  The 16 outputs at
// each edge take the direct sum: inline where the caller has registers to
// spare, out of line (kk_carrier_edge) where it has not.
__device__ __forceinline__ float2 kk_carrier_edge_inl(const float *__restrict__ mf, double r, int64_t m,
                                                      int64_t n, int64_t g0) {
  float2 tc = make_float2(0.0f, 0.0f);
#pragma unroll 1
  for (int i = 0; i < 65; i++) {
    const int64_t t = 2 * m + 32 - i;
    if (t >= 0 && t < n) tc = cadd(tc, cscale(cis_rev(-downshift_rev(r, g0 + t)), mf[i]));
  }
  return tc;
}
__device__ __noinline__ float2 kk_carrier_edge(const float *__restrict__ mf, double r, int64_t m, int64_t n,
                                               int64_t g0) {
  return kk_carrier_edge_inl(mf, r, m, n, g0);
}
__device__ __forceinline__ bool kk_interior(int64_t m, int64_t n) { return m >= 16 && 2 * m + 32 < n; }
template <bool INL = false>
__device__ __forceinline__ float2 kk_carrier_term(const RxJob &J, int64_t m, int64_t n, int64_t g0) {
  if (kk_interior(m, n)) return cmul(J.c0, cis_rev(-downshift_rev(J.r, g0 + 2 * m)));
  return INL ? kk_carrier_edge_inl(J.mf, J.r, m, n, g0) : kk_carrier_edge(J.mf, J.r, m, n, g0);
}

// KK: AGC'd carrier-free 2-sps sample u[m] = g (Z[m] - mean T[m]) (zero outside).
template <bool INL = false, class ZP>
__device__ __forceinline__ float2 kk_sample(const RxJob &J, ZP z, int64_t m, int64_t n, float2 mean, float g,
                                            int64_t g0) {
  if (m < 0 || m >= n / 2) return make_float2(0.0f, 0.0f);
  return cscale(csub(z[m], cmul(mean, kk_carrier_term<INL>(J, m, n, g0))), g);
}

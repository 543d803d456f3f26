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
// Wherever a thread's next inputs are its own previous outputs the data
// stays in registers: the codes a thread reads are the inputs of its first
// FFT butterfly, its last-pass outputs of the first transform (times H) are
// the inputs of its first butterfly of the second, and its last-pass
// outputs of the second are the phases of the samples it handles next.
#include <algorithm>
#include <type_traits>

#include "fft_lds.hpp"

__device__ __forceinline__ int64_t clamp64(int64_t v, int64_t lo, int64_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Last pass of the first transform: Y = Z H with H = -j S taken on the way
// out into registers (output k = threadIdx.x + i T of the thread goes to
// y[i], i = koff / T), the 16 spectrum weights read at the start of the pass.
template <int T> struct HilbertOut {
  const float *hspec;
  float2 (&y)[16];
  float hs[16];
  __device__ __forceinline__ void begin() {
    const int tx = tid_local();
#pragma unroll
    for (int i = 0; i < 16; i++) hs[i] = gload_u32(hspec, (unsigned)(tx + i * T));
  }
  __device__ __forceinline__ void operator()(int koff, int, float2 z) const {
    const int i = koff / T;
    y[i] = make_float2(z.y * hs[i], z.x * hs[i]);
  }
};

// Last pass of the second transform: outputs k = q + IOFF T (q = threadIdx.x
// + i T, i < QPT) are the phases phiA - j phiB of the samples the field stage
// handles; they stay in registers, in revolutions (the spectrum carries
// sgn / (2 pi)).
template <int T, int QPT, int IOFF> struct PhaseOut {
  float (&pa)[QPT];
  float (&pb)[QPT];
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ void operator()(int koff, int, float2 v) const {
    const int i = koff / T - IOFF;
    if (i >= 0 && i < QPT) {
      pa[i] = v.x;
      pb[i] = -v.y;
    }
  }
};

// The 2^14-point transforms run as 16 x 1024 (see kk_front): a wavefront's
// 1024-point transform of column k1 = its wave index hands over output
// k2 = lane + koff (slot i = koff / 64), bin k = k1 + 16 k2.
// Last pass of the first transform: times H = -j S on the way out, as
// HilbertOut, the weights read in the transform's own order.
struct HilbertOutW {
  const float *hs2;   // the column's 1024 weights, entry 64 i + lane for slot i
  float2 (&y)[16];
  float hs[16];
  __device__ __forceinline__ void begin() {
    const int lane = tid_local() & 63;
#pragma unroll
    for (int i = 0; i < 16; i++) hs[i] = gload_u32(hs2, (unsigned)(64 * i + lane));
  }
  __device__ __forceinline__ void operator()(int koff, int, float2 z) const {
    const int i = koff / 64;
    y[i] = make_float2(z.y * hs[i], z.x * hs[i]);
  }
};
// Last pass of the second transform: outputs kept in registers by slot.
struct RegOutW {
  float2 (&c)[16];
  __device__ __forceinline__ void begin() {}
  __device__ __forceinline__ void operator()(int koff, int, float2 v) const { c[koff / 64] = v; }
};

// A value that is the same in every lane, moved into scalar registers: kept
// in vector registers it would be recomputed at each use once the
// transforms have taken the register file.
__device__ __forceinline__ float2 uniform2(float2 v) {
  return make_float2(__builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v.x))),
                     __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v.y))));
}

// LDS layout of the downshifted field y' for the matched filter: planes of
// 16-bit elements with 8 elements of padding per 32 samples, so that the A
// operand of one MFMA step (8 consecutive samples of one component) is a
// single aligned 16-byte read, and the eight tiles and two planes one
// instruction reads (tile stride 20 dwords, plane offset 16 mod 64 dwords)
// fall on distinct banks.
//  PREC 0: four planes, re and im of hi = fp16(y') at 0 and PS, re and im of
//    lo = fp16(y' - hi) at 2 PS and 3 PS (the lo pair 32 mod 64 dwords on).
//  PREC 1, 2: two planes of the narrow type (re, then im PS elements on),
//    each sample rounded once when it is written.
__host__ __device__ constexpr int nidx(int q) { return q + ((q >> 5) << 3); }

// Matched-filter B operand (the tap matrix) and one wavefront pass of eight
// 16-output tiles on v_mfma_f32_16x16x32_{f16,bf16}.  Lane l holds column
// q = l % 16 and K-row group l / 16; B[t][q] = h[2 q + 64 - t] =
// htab[2 q + 95 - t] (taps h[i] at index i + 31 of a zero-padded copy in
// LDS), t = 32 ks + 8 kq + j; A[row][t] = plane[32 tile + t].
template <int PREC> struct MfB;
// The plain form keeps FP32 accuracy on the FP16 matrix pipe: each operand
// is carried as hi + lo, two FP16 values holding 22 significant bits (the
// lo part is exact: v - hi needs no rounding in FP32), and the product is
// taken as a_lo b_hi + a_hi b_lo + a_hi b_hi.  Every FP16 product is exact
// in the FP32 accumulator; the dropped a_lo b_lo is below 2^-22 of the
// term, and the split itself leaves at most 2^-22 of each operand behind,
// a few times the FP32 rounding of the sums and far below the field's own
// FP32 error.  Nine 16-cycle instructions replace the 24 32-cycle FP32
// 16x16x4 steps of the same tile pass.
template <> struct MfB<0> {
  // the lane's B vectors sit in LDS (kept in registers they would not fit
  // beside the frame-B phases): hi of step ks at bt[64 ks + lane], lo at
  // bt[192 + 64 ks + lane]; filled once per workgroup by fill()
  const rx_f16x8 *bt;
  __device__ static void fill(rx_f16x8 *tab, const float *__restrict__ mf) {
    const int tx = tid_local();
    if (tx < 192) {
      const int ks = tx >> 6, lane = tx & 63, row = lane & 15, kq = lane >> 4;
      rx_f16x8 hv, lv;
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int i = 2 * row + 64 - (32 * ks + 8 * kq + j);
        const float h = (i >= 0 && i <= 64) ? mf[i] : 0.0f;
        const _Float16 hi = (_Float16)h;
        hv[j] = hi;
        lv[j] = (_Float16)(h - (float)hi);
      }
      tab[tx] = hv;
      tab[192 + tx] = lv;
    }
  }
  __device__ void load(const rx_f16x8 *tab) { bt = tab + (tid_local() & 63); }
  // yp: this lane's component plane of hi; its lo plane is `lo` elements on
  __device__ rx_f32x4 apply(const _Float16 *__restrict__ yp, int lo, int tile, int kq) const {
    rx_f32x4 c0 = {0.0f, 0.0f, 0.0f, 0.0f}, c1 = c0;
    // nidx(32 (tile + ks) + 8 kq) = 40 (tile + ks) + 8 kq (8 kq < 32): one
    // address, the steps at immediate offsets
    const _Float16 *const a0 = yp + 40 * tile + 8 * kq;
#pragma unroll
    for (int ks = 0; ks < 3; ks++) {
      const rx_f16x8 ah = *reinterpret_cast<const rx_f16x8 *>(a0 + 40 * ks);
      const rx_f16x8 al = *reinterpret_cast<const rx_f16x8 *>(a0 + lo + 40 * ks);
      const rx_f16x8 bh = bt[64 * ks], bl = bt[192 + 64 * ks];
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, c1, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, c1, 0, 0, 0);
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, c0, 0, 0, 0);
    }
    return c0 + c1;
  }
};
template <int PREC> struct MfB {
  // precision form: operands rounded once to the narrow type
  using NT = NarrowT<PREC>;
  typename NT::vec b[3];
  __device__ void load(const float *__restrict__ htab, int row, int kq) {
#pragma unroll
    for (int ks = 0; ks < 3; ks++)
#pragma unroll
      for (int j = 0; j < 8; j++) b[ks][j] = NT::cvt(htab[2 * row + 95 - (32 * ks + 8 * kq + j)]);
  }
  // yp: this lane's component plane
  __device__ rx_f32x4 apply(const typename NT::elem *__restrict__ yp, int, int tile, int kq) const {
    rx_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const typename NT::elem *const a0 = yp + 40 * tile + 8 * kq;   // as MfB<0>::apply
#pragma unroll
    for (int ks = 0; ks < 3; ks++)
      acc = NT::mfma(*reinterpret_cast<const typename NT::vec *>(a0 + 40 * ks), b[ks], acc);
    return acc;
  }
};

// FIELD: the debug instantiation, which only writes the reconstructed field
// E of the buffers that keep it (RX_DEBUG_KEEP) and does no filtering; the
// production kernel never stores E, which keeps its registers free.
//
// Work items: item w = jb pmax + p is block pair p of launch entry jb (pairs
// past the end of a shorter buffer are skipped).  The production kernel is
// persistent: its grid is as many workgroups as the chip holds at once, each
// takes item blockIdx.x and then one item at a time from a counter in the
// scalars of launch entry 0, so a CU goes from one pair to the next without
// a workgroup dispatch in between, and workgroups that start late (their CUs
// busy with another stream's kernels) take fewer items.  The workgroup that
// finds the queue empty last resets the counters for the next launch.  The
// debug instantiation runs one workgroup per item.
// A job description read through the constant address space (its loads stay
// scalar even where the kernel has stored to global memory before them).
__device__ __forceinline__ RxJob load_job_const(const RxJob *p) {
  static_assert(sizeof(RxJob) % 4 == 0, "whole words");
  typedef const __attribute__((address_space(4))) int cword;
  const cword *src = (const cword *)p;
  RxJob j;
  int *dst = reinterpret_cast<int *>(&j);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(RxJob) / 4); i++) dst[i] = src[i];
  return j;
}

// The 16-bit words holding a thread's first-pass codes of two frames, for
// samples s0a + r T and s0b + r T (r < 16) inside the buffer: sample s sits
// at byte 3s/2 (in the high 12 bits of its word when s is odd); T is even,
// so one base per frame and immediate offsets r 3T/2.
template <int T>
__device__ __forceinline__ void front_code_words(const uint8_t *in, int64_t s0a, int64_t s0b, int (&ca)[16],
                                                 int (&cb)[16]) {
  const uint8_t *pa = in + ((3 * s0a) >> 1), *pb = in + ((3 * s0b) >> 1);
#pragma unroll
  for (int r = 0; r < 16; r++) {
    ca[r] = (int)pa[r * (3 * T / 2)] | ((int)pa[r * (3 * T / 2) + 1] << 8);
    cb[r] = (int)pb[r * (3 * T / 2)] | ((int)pb[r * (3 * T / 2) + 1] << 8);
  }
}

// Hands out a workgroup's next item: thread 0 publishes it before a barrier
// that every thread passes before reading the slot; the two parity slots keep
// the write of the item after next clear of the reads of this one.
template <bool FIELD>
__device__ __forceinline__ void front_take_next(int *nxt, int it, RxScalars *q0) {
  if (!FIELD && threadIdx.x == 0) nxt[it & 1] = (int)gridDim.x + (int)atomicAdd(&q0->kk_next, 1u);
}

// Eight per-lane doubles summed over the wavefront together: lane l returns
// the sum of variable l / 8.  Each step hands half of what a lane carries to
// a partner and adds the partner's matching half: across the two 32-lane
// halves (v[k] and v[k + 4] swapped by permlane32_swap: the low half keeps
// variable k, the high half k + 4), across pairs of 16-lane rows (the same
// with permlane16_swap), across the two 8-lane halves of a row (a DPP
// rotation by 8, one variable left), then within 8 lanes by DPP (partners
// l ^ 1, l ^ 2 and the half-row mirror).  A swap returns both registers
// rearranged; only their sum is used, which the order of the pair returned
// does not change.
template <bool ROW16>
__device__ __forceinline__ double swap_sum(double a, double b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a), ub = __builtin_bit_cast(unsigned long long, b);
  const unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32), blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
  unsigned lo0, lo1, hi0, hi1;
  if constexpr (ROW16) {
    const auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    lo0 = l[0]; lo1 = l[1]; hi0 = h[0]; hi1 = h[1];
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    lo0 = l[0]; lo1 = l[1]; hi0 = h[0]; hi1 = h[1];
  }
  return __builtin_bit_cast(double, ((unsigned long long)hi0 << 32) | lo0) +
         __builtin_bit_cast(double, ((unsigned long long)hi1 << 32) | lo1);
}
__device__ __forceinline__ double wave_sum8(const double (&v)[8], int lane) {
  double w[4], u[2];
#pragma unroll
  for (int k = 0; k < 4; k++) w[k] = swap_sum<false>(v[k], v[k + 4]);   // row R < 2: k, R >= 2: k + 4
#pragma unroll
  for (int k = 0; k < 2; k++) u[k] = swap_sum<true>(w[k], w[k + 2]);    // row R: variable 2 R + k
  const bool odd = (lane & 8) != 0;   // keeps variable 2 R + 1
  double r = (odd ? u[1] : u[0]) + dpp_f64<0x128>(odd ? u[0] : u[1]);   // row_ror:8
  r += dpp_f64<0xB1>(r);    // quad_perm [1, 0, 3, 2]
  r += dpp_f64<0x4E>(r);    // quad_perm [2, 3, 0, 1]
  r += dpp_f64<0x141>(r);   // row_half_mirror
  return r;
}

template <int LOGN, int PREC, bool FIELD = false>
__global__ __launch_bounds__((1 << LOGN) / 16, 4) void kk_front(RxLaunch L, int pmax) {  // 4 waves/SIMD: one 2^14 or two 2^13 workgroups per CU
  constexpr int N = 1 << LOGN, T = N / 16;
  constexpr int HOP = (N - RX_KK_HALFV - RX_KK_EDGE - RX_KK_CMF) & ~15;
  constexpr int QN = HOP + 2 * RX_KK_CMF;   // y' samples each block needs
  constexpr int QPT = (QN + T - 1) / T;
  constexpr int NTILE = HOP / 32;          // 16-output matched-filter tiles per block
  constexpr int NG = (NTILE + 7) / 8;      // eight tiles per wavefront pass
  constexpr int YPL = 32 * (8 * NG) + 64;  // y' samples every window of a pass reads
  static_assert(QN <= YPL && YPL % 4 == 0, "every y' sample inside the planes");
  static_assert((N / 8) % T == 0, "whole 8-sample groups per thread");
  // plane stride PS (16-bit elements, 32 mod 128); behind the narrow forms'
  // two planes, this thread's frame-B phases parked in LDS between the frames
  constexpr int PS = (YPL + 8 * ((YPL - 1) >> 5) - 32 + 127) / 128 * 128 + 32;
  static_assert(PS >= nidx(YPL - 1) + 1 && (PS + QN) * 4 <= 8 * (N + N / 16), "narrow planes and phase stash fit");
  static_assert(4 * PS * 2 <= 8 * (N + N / 16), "the plain form's four planes fit");
  // 2^14 points: the transforms as 16 x 1024, one 1024-point column per
  // wavefront in its own region of RG = fpad(1024) entries
  constexpr bool FOUR = LOGN == 14;
  constexpr int RG = fpad(1024);
  static_assert(!FOUR || 16 * RG == N + N / 16, "sixteen column regions fill the buffer");
  __shared__ float2 lds[N + N / 16];
  using ElemT = typename std::conditional<PREC == 0, _Float16, typename NarrowT<PREC == 0 ? 1 : PREC>::elem>::type;
  ElemT *const npl = reinterpret_cast<ElemT *>(lds);   // y' planes
  float *const stash = reinterpret_cast<float *>(lds) + PS;
  __shared__ double red[9 * (T / 64)];
  __shared__ float htab[128];   // matched-filter taps h[i] at i + 31, zero elsewhere
  __shared__ rx_f16x8 btab[PREC == 0 ? 384 : 1];   // the plain form's split tap operands
  __shared__ int nxt[2];   // the workgroup's next item, by iteration parity

  const int total = L.count * pmax;
  RxScalars *const q0 = FIELD ? nullptr : L.job[0]->sc;
  int it = 0;
  for (int item = blockIdx.x; item < total; it++) {
  const int jb = item / pmax;
  const int64_t pidx = item - (int64_t)jb * pmax;   // block pair of the buffer
  // the job description is never written by a kernel: read through the
  // constant address space it stays in scalar registers, although the loop
  // stores to global memory between its reads
  const RxJob J = load_job_const(L.job[jb]);
  const int64_t n = L.n[jb];
  const uint8_t *in = L.in[jb];
  const int64_t g0 = L.s0[jb] > 0 ? L.s0[jb] : 0;   // stream index of sample 0 (downshift phase)
  const int64_t nrb = (n + HOP - 1) / HOP;
  const int64_t blk[2] = {2 * pidx, 2 * pidx + 1};
  if (blk[0] >= nrb || (FIELD && !J.field)) {
    front_take_next<FIELD>(nxt, it, q0);
    __syncthreads();
  } else {
  const int64_t F[2] = {blk[0] * HOP - RX_KK_EDGE, blk[1] * HOP - RX_KK_EDGE};
  if (!FIELD && pidx == 0 && threadIdx.x == 0) J.sc->t_start = (unsigned long long)wall_clock64();   // buffer start

  if constexpr (PREC == 0) {
    MfB<0>::fill(btab, J.mf);
  } else if (tid_local() < 128) {
    const int tx = tid_local(), i = tx - 31;
    htab[tx] = (i >= 0 && i <= 64) ? J.mf[i] : 0.0f;
  }

  // 1. log2 v - log2 v_ref for both frames (v_ref: the frame's centre
  //    sample; the Hilbert response is zero at DC, so any offset leaves phi
  //    unchanged and a small one keeps the FP32 transform accurate), with
  //    v = code + 0.5 in [0.5, 4095.5], so the hardware log2 (1 ulp) needs
  //    none of the denormal handling of logf.  l = ln(sqrt(v)) is
  //    (ln 2 / 2) log2 v: the transforms are linear, so that factor (and
  //    1 / (2 pi) for a phase in revolutions) rides in the spectrum weights.
  //    Taken straight into the first FFT pass (radix 16, no twiddles):
  //    butterfly j = threadIdx.x reads samples j + r T (r < 16), so the thread
  //    reads those codes itself, transforms them in registers and writes the
  //    pass's outputs 16 j + r; the codes never pass through LDS.
  // The field stage's samples t = F + EDGE - CMF + q, q = j + i T, are this
  // thread's first-pass samples r = i + IOFF of the same frame: their codes
  // stay in registers (both frames' 12-bit codes packed in one word).
  static_assert((RX_KK_EDGE - RX_KK_CMF) % T == 0 && QN % T == 0, "phases are the thread's own outputs");
  constexpr int IOFF = (RX_KK_EDGE - RX_KK_CMF) / T;
  static_assert(QPT + IOFF <= 16, "the field stage's codes are first-pass codes");
  int cpk[QPT];
  const float lr0 = __builtin_amdgcn_logf((float)read_code(in, clamp64(F[0] + N / 2, 0, n - 1)) + 0.5f);
  const float lr1 = __builtin_amdgcn_logf((float)read_code(in, clamp64(F[1] + N / 2, 0, n - 1)) + 0.5f);
  {
    const int tx = tid_local();
    int ca[16], cb[16];
    if (F[0] >= 0 && F[1] + N <= n) {
      // both frames inside the buffer: sample s0 + r T sits at byte
      // (3 s0 >> 1) + r (3 T / 2) (T is even), in the high 12 bits of its
      // 16-bit word when s0 is odd
      const int64_t s0a = F[0] + tx, s0b = F[1] + tx;
      const int sha = (int)(s0a & 1) << 2, shb = (int)(s0b & 1) << 2;
      front_code_words<T>(in, s0a, s0b, ca, cb);
#pragma unroll
      for (int r = 0; r < 16; r++) {
        ca[r] = (ca[r] >> sha) & 0xFFF;
        cb[r] = (cb[r] >> shb) & 0xFFF;
      }
    } else {   // a frame reaches past a buffer end: samples replicated from the edge
#pragma unroll
      for (int r = 0; r < 16; r++) {
        ca[r] = read_code(in, clamp64(F[0] + tx + r * T, 0, n - 1));
        cb[r] = read_code(in, clamp64(F[1] + tx + r * T, 0, n - 1));
      }
    }
    float2 w1, w2, w4, w8;   // W^(j r) of the 16 x 1024 form's first step, read beside the codes
    if constexpr (FOUR) {
      const GView2 tg = gview(J.twid);
      w1 = tg.at(tx);
      w2 = tg.at(2 * tx);
      w4 = tg.at(4 * tx);
      w8 = tg.at(8 * tx);
    }
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; r++)
      v[r] = make_float2(__builtin_amdgcn_logf((float)ca[r] + 0.5f) - lr0,
                         __builtin_amdgcn_logf((float)cb[r] + 0.5f) - lr1);
#pragma unroll
    for (int i = 0; i < QPT; i++) cpk[i] = ca[i + IOFF] | (cb[i + IOFF] << 16);
    front_take_next<FIELD>(nxt, it, q0);   // its latency overlaps the code reads
    dft16(v);
    if constexpr (FOUR) {
      // output k1 = r, times W_N^(j k1), to column k1: G[k1][j] at k1 RG + j
      apply_twiddles<16, 1>(v, w1, w2, w4, w8);
#pragma unroll
      for (int r = 0; r < 16; r++) lds[r * RG + tx] = v[r];
    } else {
      const int p0 = fpad(16 * tx);   // outputs 16 j + r: one padded run
#pragma unroll
      for (int r = 0; r < 16; r++) lds[p0 + r] = v[r];
    }
  }
  __syncthreads();

  // 2. Hilbert filtering: Y = Z H, H = -j S; the inverse transform is done as
  //    conj(FFT(conj(Y)/N)), so the second pass leaves phiA - j phiB.  Each
  //    thread's outputs of either transform (k = threadIdx.x mod T) are the
  //    ones it multiplies by H and, after the second, the phases of the
  //    samples it handles in the field stage (q + EDGE - CMF with q =
  //    threadIdx.x + i T): both are taken in the last pass, in registers.
  //    The first pass of the second transform (radix 16, no twiddles) takes,
  //    for butterfly j = threadIdx.x, inputs j + r T: the thread's own
  //    Hilbert products, so they go from one transform to the other in
  //    registers; the barrier only keeps the writes behind every thread's
  //    reads of the last pass.
  // the phases come out as sgn phi / (2 pi), in revolutions: the spectrum
  // weights carry sgn (ln 2 / 2) / (2 pi)
  float ph[2][QPT];   // frames A and B (the narrow forms park B in LDS below)
  if constexpr (FOUR) {
    // 16 x 1024: X[k1 + 16 k2] = sum_j W_1024^(j k2) W_N^(j k1) sum_r x[j + T r]
    // W_16^(r k1).  The inner sums and twiddles are done (thread j, above);
    // wavefront k1 now takes column k1 (lane l: j = l + 64 m) and
    // transforms it in its own LDS region, with wavefront-local exchanges
    // only.  The second transform runs the same steps in reverse order:
    // Z[m2 + T m1] = sum_k1 W_16^(m1 k1) W_N^(m2 k1) sum_k2 c[k1 + 16 k2]
    // W_1024^(m2 k2), with c = conj(Y) the column's own products, so only
    // its last step (thread m2 = j, all k1) needs the workgroup again.
    static_assert(N == 16 * 1024 && T == 1024 && QPT + IOFF <= 16, "16 x 1024 geometry");
    const int lane = tid_local() & 63, wv = tid_local() >> 6;
    float2 *const wb = lds + wv * RG;
    const float2 *const tw1k = J.twid + N;
    float2 y[16];
    {
      float2 x[16];
#pragma unroll
      for (int m = 0; m < 16; m++) x[m] = wb[64 * m + lane];
      wave_sync();
      dft16(x);   // first pass of the column transform (radix 16, no twiddles)
      const int p0 = fpad(16 * lane);
#pragma unroll
      for (int r = 0; r < 16; r++) wb[p0 + r] = x[r];
    }
    wave_sync();
    fft_passes<1024, 16, false, HilbertOutW, false, true>(wb, tw1k, HilbertOutW{J.hspec + N + 1024 * wv, y, {}});
    // second transform: the column's products are its first pass's inputs
    // (slot m' = element lane + 64 m')
    dft16(y);
    wave_sync();
    {
      const int p0 = fpad(16 * lane);
#pragma unroll
      for (int r = 0; r < 16; r++) wb[p0 + r] = y[r];
    }
    wave_sync();
    float2 c[16];
    fft_passes<1024, 16, false, RegOutW, false, true>(wb, tw1k, RegOutW{c});
    // element m2 = lane + 64 m of column k1 = wv to thread m2: G[m][wv][lane]
    const int tx = tid_local();
    const GView2 tg = gview(J.twid);
    const float2 u1 = tg.at(tx), u2 = tg.at(2 * tx), u4 = tg.at(4 * tx), u8 = tg.at(8 * tx);
    __syncthreads();   // every wavefront is done with its region
#pragma unroll
    for (int m = 0; m < 16; m++) lds[m * RG + 64 * wv + lane] = c[m];
    __syncthreads();
    float2 z[16];
#pragma unroll
    for (int k1 = 0; k1 < 16; k1++) z[k1] = lds[wv * RG + 64 * k1 + lane];
    apply_twiddles<16, 1>(z, u1, u2, u4, u8);   // W_N^(j k1)
    dft16(z);   // z[m1] = output j + T m1
#pragma unroll
    for (int i = 0; i < QPT; i++) {
      ph[0][i] = z[i + IOFF].x;
      ph[1][i] = -z[i + IOFF].y;
    }
  } else {
    {
      float2 y[16];
      fft_passes<N, 16, false>(lds, J.twid, HilbertOut<T>{J.hspec, y, {}});   // the passes after the first
      dft16(y);
      __syncthreads();
      const int p0 = fpad(16 * tid_local());   // outputs 16 j + r of the second transform's first pass
#pragma unroll
      for (int r = 0; r < 16; r++) lds[p0 + r] = y[r];
    }
    __syncthreads();
    // the second transform recomputes its twiddle addresses: kept live from
    // the first they would be spilled across the Hilbert product
    const float2 *tw2 = J.twid;
    asm volatile("" : "+s"(tw2));
    fft_passes<N, 16, false>(lds, tw2, PhaseOut<T, QPT, IOFF>{ph[0], ph[1]});
  }
  // the phases are formed here: left to itself the compiler moves the last
  // pass's arithmetic into the field stage, where it no longer fits the
  // register file
#pragma unroll
  for (int i = 0; i < QPT; i++) asm volatile("" : "+v"(ph[0][i]), "+v"(ph[1][i]));
  __syncthreads();
  if constexpr (PREC != 0) {
    const int tx = tid_local();
#pragma unroll
    for (int i = 0; i < QPT; i++) {
      const int q = tx + i * T;
      stash[q] = ph[1][i];   // read back by this thread only
    }
  }

  // Workgroup partial sums: the field E (carrier mean), |Z|^2, and the
  // carrier terms.  In the interior T[m] = c0 P(m)^*, P(m) = exp(+j 2 pi
  // frac(2 r m)), so sum Z conj(T) = conj(c0) sum Z P and sum |T|^2 = |c0|^2
  // per output; the edge outputs take the exact T.  Per-thread sums are in
  // FP32 (at most a few dozen terms), the workgroup sums in FP64.
  float se_re = 0.0f, se_im = 0.0f, zz = 0.0f;
  float2 sp = make_float2(0.0f, 0.0f), sedge = make_float2(0.0f, 0.0f);
  float tedge = 0.0f;
  // interior outputs of the workgroup's two blocks (a count fixed by the
  // geometry, workgroup-uniform)
  int nint = 0;
  const int lane = tid_local() & 63, wv = tid_local() >> 6;
  const int row = lane & 15, kq = lane >> 4;
  constexpr int NW = T / 64;
  // rotations of P between this lane's outputs: +16 (second tile) and
  // +16 * 8 * NW (next pass)
  const float2 r16 = uniform2(cis_rev(downshift_rev(J.r, 2 * 16)));
  const float2 rpass = uniform2(cis_rev(downshift_rev(J.r, 2 * 16 * 8 * NW)));
  const float2 drot = uniform2(cis_rev(-downshift_rev(J.r, T)));   // downshift phasor step over T samples
#pragma unroll
  for (int x = 0; x < 2; x++) {
    // 3. field, carrier mean partials, downshifted field y' = E D into LDS.
    //    This thread's samples t = nq0 + q, q = threadIdx + i T, are T apart,
    //    so the downshift phasor D(t) = exp(-j 2 pi frac(r t)) starts from an
    //    FP64 anchor and advances by the fixed rotation D(T) per sample.
    //    Their codes are the first pass's (clamped into the buffer there;
    //    samples outside it give y' = 0 here).
    const int64_t nq0 = F[x] + RX_KK_EDGE - RX_KK_CMF;   // sample index of q = 0
    const int qlo = (int)clamp64(-nq0, 0, QN), qhi = (int)clamp64(n - nq0, 0, QN);   // t in [0, n)
    // interior frames (all samples inside the buffer: every block pair but
    // a buffer's first and last) skip the range masks
    const bool inner = __builtin_amdgcn_readfirstlane((int)(qlo == 0 && qhi == QN)) != 0;
    const int tx = tid_local();
    float2 dph = cis_rev(-downshift_rev(J.r, g0 + nq0 + tx));
    float2 *const fbase = J.field + nq0;   // FIELD only
    // plane index of q = tx + i T: nidx(tx) + nidx(i T), T a multiple of 32
    static_assert(T % 32 == 0, "plane offsets split");
    const int nq = nidx(tx);
    // the LDS offset field holds 16 bits: the two lo planes take bases of
    // their own, formed once, with the sample's offset as the immediate
    int nq2 = nq + 2 * PS, nq3 = nq + 3 * PS;
    asm volatile("" : "+v"(nq2), "+v"(nq3));
#pragma unroll
    for (int i = 0; i < QPT; i++) {
      const int q = tx + i * T;   // < QN: QN is a multiple of T
      const int c = x == 0 ? (cpk[i] & 0xFFF) : (cpk[i] >> 16);
      float phv;
      if constexpr (PREC == 0) phv = ph[x][i];
      else phv = x == 0 ? ph[0][i] : stash[q];
      // sqrt(v): v in [0.5, 4095.5], so the hardware square root (1 ulp)
      // needs none of the denormal or rounding fix-ups of sqrtf
      float2 ev = cscale(cis_rev(phv), __builtin_amdgcn_sqrtf((float)c + 0.5f));
      float2 yv = cmul(ev, dph);
      if (!inner) {
        if (q < qlo || q >= qhi) {
          ev = make_float2(0.0f, 0.0f);
          yv = ev;
        }
      }
      if (q >= RX_KK_CMF && q < RX_KK_CMF + HOP) {
        se_re += ev.x;
        se_im += ev.y;
        if constexpr (FIELD) {
          if (q >= qlo && q < qhi) gstore(fbase, q, ev);
        }
      }
      const int pq = nq + nidx(i * T);
      if constexpr (FIELD) {
      } else if constexpr (PREC == 0) {
        // both components converted as one pair (the same rounding as
        // one at a time); lo = y - hi, exact in FP32, rounded once to FP16
        // by a mixed-precision FMA (hi as its FP16 operand, -1, y)
        const rx_f32x2 y2 = {yv.x, yv.y};
        const rx_f16x2 hi = __builtin_convertvector(y2, rx_f16x2);
        const unsigned hb = __builtin_bit_cast(unsigned, hi);
        unsigned lb;
        asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(lb) : "v"(hb), "v"(y2.x));
        asm("v_fma_mixhi_f16 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(lb) : "v"(hb), "v"(y2.y));
        const rx_f16x2 lo = __builtin_bit_cast(rx_f16x2, lb);
        npl[pq] = hi.x;
        npl[PS + pq] = hi.y;
        npl[nq2 + nidx(i * T)] = lo.x;
        npl[nq3 + nidx(i * T)] = lo.y;
      } else {
        npl[pq] = NarrowT<PREC == 0 ? 1 : PREC>::cvt(yv.x);
        npl[PS + pq] = NarrowT<PREC == 0 ? 1 : PREC>::cvt(yv.y);
      }
      dph = cmul(dph, drot);
    }
    if constexpr (FIELD) continue;
    __syncthreads();
    // 4. decimating matched filter Z[m] = sum_i h[i] y'[2m + 32 - i] as a
    //    Toeplitz GEMM on MFMA: a row of A is one real component (re or im)
    //    of the 96-sample window of a tile of 16 outputs, B[t][q] =
    //    h[2q + 64 - t]; eight tiles (16 rows) per wavefront pass, 16x16x32
    //    steps with FP32 accumulation: PREC 0 on split (hi + lo) FP16
    //    operands, the precision form on operands rounded to the narrow type.
    // the next item (published before this pair's first barrier): one read
    // per 128-byte line of its input brings that into this CU's L2 while
    // this matched filter runs, so the next pair's first reads hit there
    unsigned warm = 0;
    if constexpr (!FIELD) {
      if (x == 1) {
        const int nit = __builtin_amdgcn_readfirstlane(nxt[it & 1]);
        if (nit < total) {
          const int njb = nit / pmax;
          const int64_t np = nit - (int64_t)njb * pmax, nn = L.n[njb];
          const int64_t nF0 = 2 * np * HOP - RX_KK_EDGE;
          if (2 * np < (nn + HOP - 1) / HOP) {
            // samples [lo, hi) of its two frames inside the buffer (all even)
            const int64_t lo = nF0 > 0 ? nF0 : 0, hi = nF0 + HOP + N < nn ? nF0 + HOP + N : nn;
            const int64_t b0 = (3 * lo / 2) & ~(int64_t)3, off = b0 + 128 * (int64_t)tid_local();
            if (off + 4 <= 3 * hi / 2) warm = *gptr(reinterpret_cast<const uint32_t *>(L.in[njb] + off));
          }
        }
      }
    }
    const int64_t m0 = blk[x] * (HOP / 2);
    MfB<PREC> bmf;
    if constexpr (PREC == 0) bmf.load(btab);
    else bmf.load(htab, row, kq);
    // P at this lane's first output of the block, exact from the FP64 phase
    const int64_t mfirst = m0 + 16 * (8 * wv + 2 * kq) + row;
    float2 pp = cis_rev(downshift_rev(J.r, g0 + 2 * mfirst));
    // outputs are handled by their offset mr = m - m0 < HOP / 2 in the block:
    // valid (2 m < n) below mlim, interior (m >= 16, 2 m + 32 < n) in
    // [mil, mih); n is even, so both limits are exact integers
    const int mlim = (int)clamp64(n / 2 - m0, 0, HOP / 2);
    const int mil = (int)clamp64(16 - m0, 0, HOP / 2);
    const int mih = (int)clamp64((n - 32) / 2 - m0, 0, HOP / 2);
    nint += mih > mil ? mih - mil : 0;
    float2 *const zb = J.z + m0;
    for (int grp = wv; grp < NG; grp += NW) {
      const int tile = grp * 8 + (row >> 1);
      rx_f32x4 acc;
      acc = bmf.apply(npl + (row & 1) * PS, 2 * PS, tile, kq);
#pragma unroll
      for (int jj = 0; jj < 2; jj++) {
        const int t2 = grp * 8 + 2 * kq + jj;
        const int mr = 16 * t2 + row;
        const float2 p = jj ? cmul(pp, r16) : pp;
        if (t2 < NTILE && mr < mlim) {
          const float2 zv = make_float2(acc[2 * jj], acc[2 * jj + 1]);
          gstore_u32(zb, (unsigned)mr, zv);
          zz = fmaf(zv.x, zv.x, fmaf(zv.y, zv.y, zz));
          if (mr >= mil && mr < mih) {
            sp = cadd(sp, cmul(zv, p));
          } else {
            const float2 te = kk_carrier_edge_inl(J.mf, J.r, m0 + mr, n, g0);
            sedge = cadd(sedge, cmulc(zv, te));
            tedge = fmaf(te.x, te.x, fmaf(te.y, te.y, tedge));
          }
        }
      }
      pp = cmul(pp, rpass);
    }
    asm volatile("" : : "v"(warm));   // the warming read has landed by now
    // the second frame's reads of the planes are kept from the next pair's
    // writes by the barrier of the workgroup sums below
    if (x == 0) __syncthreads();
  }
  if constexpr (!FIELD) {
  // FP64 workgroup sums of eight variables: each wavefront's at once
  // (wave_sum8: variable s in lanes 8 s .. 8 s + 7), then lane s < 8 of the
  // first wavefront adds variable s over the wavefronts in wavefront order
  // and thread 0 collects them; only thread 0 needs them.  The edge sums
  // are zero outside the edge workgroups, the interior count is nint.
  const double w8[8] = {se_re, se_im, zz, tedge, sp.x, sp.y, sedge.x, sedge.y};
  const double ws = wave_sum8(w8, lane);
  if ((lane & 7) == 0) red[(lane >> 3) * NW + wv] = ws;
  __syncthreads();
  if (wv == 0) {
    double sk = 0.0;
    if (lane < 8)
      for (int i = 0; i < NW; i++) sk += red[lane * NW + i];
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; k++) v[k] = __shfl(sk, k);
    if (lane == 0) {
      const double c0r = J.c0.x, c0i = J.c0.y;
      J.part[3 * pidx] = make_double2(v[0], v[1]);                          // sum of the field E
      J.part[3 * pidx + 1] = make_double2(v[2], v[3] + (double)nint * (c0r * c0r + c0i * c0i));  // |Z|^2, |T|^2
      J.part[3 * pidx + 2] = make_double2(c0r * v[4] + c0i * v[5] + v[6],    // sum Z conj(T)
                                          c0r * v[5] - c0i * v[4] + v[7]);
    }
  }
  }
  }
  if constexpr (FIELD) break;
  item = __builtin_amdgcn_readfirstlane(nxt[it & 1]);
  }
  // every workgroup's last take came back empty before it counts itself
  // here, so the last one to count resets the queue for the next launch
  if (!FIELD && threadIdx.x == 0 && atomicAdd(&q0->kk_done, 1u) == gridDim.x - 1) {
    atomicExch(&q0->kk_next, 0u);
    atomicExch(&q0->kk_done, 0u);
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
  J.udbg[m] = kk_sample(J, J.z, m, n, mean, (float)J.sc->agc, L.s0[jb] > 0 ? L.s0[jb] : 0);
}

// Viterbi-Viterbi carrier phase per DD-LMS block over blocks b-1..b+1,
// unwrapped in multiples of pi/2 (wrapped differences, then a workgroup
// prefix sum), one workgroup per buffer.  A stream buffer after the first
// continues the unwrap from the phase carried from the previous buffer's
// last emitted block (the block just before its first emitted one), and
// every stream buffer carries its own last emitted block's phase on.
__global__ __launch_bounds__(1024) void kk_vv(RxLaunch L) {
  __shared__ double scan[1024];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int64_t nsym = n / 4;
  const int nb = (int)(nsym / J.blk);
  if (J.dd_phase) {   // the DD-LMS taps carry the phase: no derotation
    for (int b = threadIdx.x; b < nb; b += 1024) J.theta[b] = 0.0f;
    return;
  }
  const RxSpan sp = rx_span(J, n, L.s0[jb]);
  const bool cont = J.stream && L.s0[jb] >= 0;
  const int bs = cont ? (int)(sp.k_lo / J.blk) - 1 : 0;   // first block of the scan
  const int blast = (int)(sp.k_hi / J.blk) - 1;            // last emitted block
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
  const double first = cont ? J.sc->theta_carry : 0.0;
  auto step = [&](int b, float r, float prev) -> double {
    if (b < bs) return 0.0;
    if (b == bs) return cont ? first : (double)r;
    return wrapq(r - prev);
  };
  double local = 0.0;
  float prev = (b0 > 0 && b0 < nb) ? raw(b0 - 1) : 0.0f;
  for (int b = b0; b < b0 + per && b < nb; b++) {
    const float r = raw(b);
    local += step(b, r, prev);
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
    th += step(b, r, prev);
    prev = r;
    J.theta[b] = (float)th;
    if (J.stream && b == blast) J.sc->theta_carry = th;
  }
}

// The persistent grid: as many workgroups as the device holds at once.
template <int LOGN, int PREC>
static int front_resident() {
  static int resident = 0;   // one device type per process
  if (resident == 0) {
    int dev = 0, ncu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kk_front<LOGN, PREC, false>, (1 << LOGN) / 16, 0) !=
            hipSuccess)
      return 256;
    resident = ncu * (occ > 0 ? occ : 1);
  }
  return resident;
}

template <int LOGN, int PREC, bool FIELD = false>
static void launch_front(const RxLaunch &L, int64_t maxn, hipStream_t s) {
  constexpr int N = 1 << LOGN;
  const int hop = rx_kk_hop(LOGN);
  const int64_t nrb = (maxn + hop - 1) / hop;
  const int pmax = (int)((nrb + 1) / 2);
  const int64_t total = (int64_t)pmax * L.count;
  if (total <= 0) return;
  const int64_t grid = FIELD ? total : std::min<int64_t>(total, front_resident<LOGN, PREC>());
  hipLaunchKernelGGL((kk_front<LOGN, PREC, FIELD>), dim3((unsigned)grid), dim3(N / 16), 0, s, L, pmax);
}

void rx_launch_kk_stage(int stage, const RxLaunch &L, int64_t maxn, int log2n, int prec, hipStream_t s) {
  const unsigned cnt = (unsigned)L.count;
  if (stage == ST_KK_FRONT) {
    if (log2n == RX_KK_FD_LOG2) {
      rx_launch_kkfd(L, maxn, s);
    } else if (log2n == 13) {
      if (prec == 1) launch_front<13, 1>(L, maxn, s);
      else if (prec == 2) launch_front<13, 2>(L, maxn, s);
      else launch_front<13, 0>(L, maxn, s);
    } else {
      if (prec == 1) launch_front<14, 1>(L, maxn, s);
      else if (prec == 2) launch_front<14, 2>(L, maxn, s);
      else launch_front<14, 0>(L, maxn, s);
    }
  } else if (stage == ST_KK_DEBUG) {
    // the field E (the same FP32 arithmetic in every form; the
    // frequency-domain front end writes it itself), then u
    if (log2n == 13) launch_front<13, 0, true>(L, maxn, s);
    else if (log2n == 14) launch_front<14, 0, true>(L, maxn, s);
    const int64_t nd = maxn / 2;
    hipLaunchKernelGGL(kk_debug_u, dim3((unsigned)((nd + 255) / 256), cnt), dim3(256), 0, s, L);
  } else if (stage == ST_KK_VV) {
    hipLaunchKernelGGL(kk_vv, dim3(1, cnt), dim3(1024), 0, s, L);
  }
}

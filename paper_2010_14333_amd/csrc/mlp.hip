// Learned equaliser for the PAM chain: an MLP 31 -> 64 ReLU -> 64 ReLU -> 1
// over 31 timing-corrected samples centred on each symbol, used in place of
// the block DD-LMS FFE (the paper equalises with an LMS FFE, Sec. 2 ¶1; the
// network replaces it on nonlinear links).  Training: FP32 forward,
// backward and Adam (Kingma & Ba 2015) kernels.  Inference: BF16 operands on
// MFMA with FP32 accumulation.  Parameters are packed W1[64][31], b1[64],
// W2[64][64], b2[64], W3[64], b3.
#include <map>
#include <mutex>

#include "fft_lds.hpp"   // rx_dev.hpp and wave_sync

#define MI 31
#define MH 64
#define MP (MH * MI + MH + MH * MH + MH + MH + 1)
#define OFF_B1 (MH * MI)
#define OFF_W2 (OFF_B1 + MH)
#define OFF_B2 (OFF_W2 + MH * MH)
#define OFF_W3 (OFF_B2 + MH)
#define OFF_B3 (OFF_W3 + MH)
#define SPW 64   // samples per workgroup in the training kernels

// ---- training -------------------------------------------------------------
// Partial gradient of the minibatch loss (1/B) sum (y - t)^2 over the SPW
// samples of this workgroup.  Sample e of the minibatch is row
// (mult * (i0 + e)) mod ntrain of the training set (mult coprime to ntrain:
// a permutation per epoch), or row e when mult == 0.
__global__ __launch_bounds__(256) void mlp_grad_partial(const float *__restrict__ p, const float *__restrict__ X,
                                                        const float *__restrict__ Tg, int64_t ntrain, int64_t i0,
                                                        int batch, int64_t mult, float *__restrict__ part,
                                                        double *__restrict__ loss_part) {
  __shared__ float w[MP];
  __shared__ float xs[SPW][32];
  __shared__ float h1[SPW][MH + 1], h2[SPW][MH + 1], d1[SPW][MH + 1], d2[SPW][MH + 1];
  __shared__ float dy[SPW], tt[SPW];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  for (int i = tid; i < MP; i += 256) w[i] = p[i];
  const int e0 = blockIdx.x * SPW;
  for (int i = tid; i < SPW * 32; i += 256) {
    const int sidx = i / 32, c = i % 32, e = e0 + sidx;
    float v = 0.0f;
    if (e < batch && c < MI) {
      const int64_t row = mult ? (int64_t)(((uint64_t)mult * (uint64_t)(i0 + e)) % (uint64_t)ntrain) : e;
      v = X[row * 32 + c];
    }
    xs[sidx][c] = v;
  }
  if (tid < SPW) {
    const int e = e0 + tid;
    const int64_t row = (e < batch) ? (mult ? (int64_t)(((uint64_t)mult * (uint64_t)(i0 + e)) % (uint64_t)ntrain) : e) : 0;
    tt[tid] = (e < batch) ? Tg[row] : 0.0f;
  }
  __syncthreads();
  // layer 1 and 2 forward: thread -> 16 (sample, unit) pairs
  for (int q = tid; q < SPW * MH; q += 256) {
    const int sidx = q / MH, o = q % MH;
    float a = 0.0f;
    for (int i = 0; i < MI; i++) a = fmaf(w[o * MI + i], xs[sidx][i], a);
    a += w[OFF_B1 + o];
    h1[sidx][o] = a > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  for (int q = tid; q < SPW * MH; q += 256) {
    const int sidx = q / MH, o = q % MH;
    float a = 0.0f;
    for (int i = 0; i < MH; i++) a = fmaf(w[OFF_W2 + o * MH + i], h1[sidx][i], a);
    a += w[OFF_B2 + o];
    h2[sidx][o] = a > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  double lp = 0.0;
  if (tid < SPW) {
    float a = w[OFF_B3];
    for (int i = 0; i < MH; i++) a = fmaf(w[OFF_W3 + i], h2[tid][i], a);
    const bool live = e0 + tid < batch;
    const float r = live ? a - tt[tid] : 0.0f;
    lp = (double)r * r;
    dy[tid] = 2.0f * r / (float)batch;
  }
  __syncthreads();
  for (int q = tid; q < SPW * MH; q += 256) {
    const int sidx = q / MH, o = q % MH;
    d2[sidx][o] = h2[sidx][o] > 0.0f ? dy[sidx] * w[OFF_W3 + o] : 0.0f;
  }
  __syncthreads();
  for (int q = tid; q < SPW * MH; q += 256) {
    const int sidx = q / MH, i = q % MH;
    float a = 0.0f;
    for (int o = 0; o < MH; o++) a = fmaf(w[OFF_W2 + o * MH + i], d2[sidx][o], a);
    d1[sidx][i] = h1[sidx][i] > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  // parameter gradients summed over this workgroup's samples
  float *out = part + (int64_t)blockIdx.x * MP;
  for (int q = tid; q < MP; q += 256) {
    float g = 0.0f;
    if (q < OFF_B1) {
      const int o = q / MI, i = q % MI;
      for (int sidx = 0; sidx < SPW; sidx++) g = fmaf(d1[sidx][o], xs[sidx][i], g);
    } else if (q < OFF_W2) {
      for (int sidx = 0; sidx < SPW; sidx++) g += d1[sidx][q - OFF_B1];
    } else if (q < OFF_B2) {
      const int o = (q - OFF_W2) / MH, i = (q - OFF_W2) % MH;
      for (int sidx = 0; sidx < SPW; sidx++) g = fmaf(d2[sidx][o], h1[sidx][i], g);
    } else if (q < OFF_W3) {
      for (int sidx = 0; sidx < SPW; sidx++) g += d2[sidx][q - OFF_B2];
    } else if (q < OFF_B3) {
      for (int sidx = 0; sidx < SPW; sidx++) g = fmaf(dy[sidx], h2[sidx][q - OFF_W3], g);
    } else {
      for (int sidx = 0; sidx < SPW; sidx++) g += dy[sidx];
    }
    out[q] = g;
  }
  lp = block_sum(lp, red);
  if (tid == 0) loss_part[blockIdx.x] = lp;
}

// Sum of the partial gradients; with adam != 0 also the Adam update
// (bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t from the host).
__global__ __launch_bounds__(256) void mlp_reduce_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                                                       const float *__restrict__ part, int nparts, float *__restrict__ grad,
                                                       int adam, float lr, float b1, float b2, float eps, float c1,
                                                       float c2) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= MP) return;
  float g = 0.0f;
  for (int i = 0; i < nparts; i++) g += part[(int64_t)i * MP + q];
  if (grad) grad[q] = g;
  if (adam) {
    const float mm = b1 * m[q] + (1.0f - b1) * g;
    const float vv = b2 * v[q] + (1.0f - b2) * g * g;
    m[q] = mm;
    v[q] = vv;
    p[q] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// Training rows of one processed buffer: for symbols k in [64, nsym - 64),
// X = xr[2(k+s) - 15 .. 2(k+s) + 15] (zero outside, column 31 zero) and
// T = the transmitted level of symbol k.
__global__ __launch_bounds__(256) void mlp_windows(RxLaunch L, float *__restrict__ X, float *__restrict__ Tg,
                                                   int64_t row0) {
  const RxJob J = *L.job[0];
  const int64_t n = L.n[0], nsym = n / 2;
  const int64_t k = RX_GUARD + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= nsym - RX_GUARD) return;
  const int s = J.sc->lag;
  const int64_t row = row0 + (k - RX_GUARD);
  const int64_t c = 2 * (k + s) - 15;
  for (int i = 0; i < 32; i++) {
    const int64_t j = c + i;
    X[row * 32 + i] = (i < MI && j >= 0 && j < n) ? J.xr[j] : 0.0f;
  }
  Tg[row] = ref_symbol(J, k).x;
}

// ---- inference (BF16 MFMA) -----------------------------------------------
// Per wavefront, tiles of 16 symbols (v_mfma_f32_16x16x32_bf16: lane l
// supplies A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16] and
// receives D[4 (l / 16) + j][l % 16]):
//   layer 1: H1^T (64 x 16) = W1 (64 x 32) X^T (32 x 16) + b1: 4 MFMA, the
//            bias as the accumulator input;
//   layer 2: H2^T = W2 (64 x 64) H1^T + b2: 8 MFMA.  Lane l holds after layer
//            1 the units 16 t + 4 kq + j (kq = l / 16, t, j < 4) of symbol
//            l % 16, so layer 2 takes its K index in the order
//            u(ks, kq, jj) = 16 (2 ks + jj / 4) + 4 kq + jj % 4 (W2's columns
//            permuted to match) and the ReLU'd layer-1 outputs become its B
//            operand without leaving the registers;
//   layer 3: y = W3 . H2 + b3: 2 MFMA with W3 in row 0 of A (the other
//            rows zero) and the ReLU'd layer-2 outputs as B in the same K
//            order, so lane l < 16 receives y of symbol l.
#define TILES_PER_WAVE 64   // amortises loading the network into registers (training-side rows)
// the chain's inference: a wavefront's set-up (the network's fragments
// converted into registers and LDS) is paid once per this many tiles
#define MLP_INFER_TPW 256
using MNT = NarrowT<1>;

struct MlpFrag {
  MNT::vec a1[4], a2[4][2];   // A fragments: W1 row tiles, W2 row tiles x 2 K-steps (permuted)
  MNT::vec a3[2];             // W3 in row 0 (lanes l % 16 == 0), 2 K-steps in layer 2's order
  const float *cv;            // LDS: b1[64], b2[64] (the biases, read per tile)
  const MNT::vec *a2l;        // or the W2 fragments in LDS, [t][ks][lane] (then a2 is unused)
  float b3;
};

// Every thread of the workgroup calls this (it fills the LDS vectors, and
// the W2 fragments into a2l when that is given).
__device__ __forceinline__ void mlp_load_frag(const float *__restrict__ P, int row, int kq, float *cv, MlpFrag &f,
                                              MNT::vec *a2l = nullptr) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int jj = 0; jj < 8; jj++) {
      const int i = 8 * kq + jj;
      f.a1[t][jj] = MNT::cvt(i < MI ? P[(16 * t + row) * MI + i] : 0.0f);
      if (!a2l) {
#pragma unroll
        for (int ks = 0; ks < 2; ks++) {
          const int u = 16 * (2 * ks + jj / 4) + 4 * kq + jj % 4;
          f.a2[t][ks][jj] = MNT::cvt(P[OFF_W2 + (16 * t + row) * MH + u]);
        }
      }
    }
#pragma unroll
  for (int ks = 0; ks < 2; ks++)
#pragma unroll
    for (int jj = 0; jj < 8; jj++) {
      const int u = 16 * (2 * ks + jj / 4) + 4 * kq + jj % 4;
      f.a3[ks][jj] = MNT::cvt(row == 0 ? P[OFF_W3 + u] : 0.0f);
    }
  if (a2l && threadIdx.x < 64) {
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int ks = 0; ks < 2; ks++) {
        MNT::vec v;
#pragma unroll
        for (int jj = 0; jj < 8; jj++) {
          const int u = 16 * (2 * ks + jj / 4) + 4 * kq + jj % 4;
          v[jj] = MNT::cvt(P[OFF_W2 + (16 * t + row) * MH + u]);
        }
        a2l[(2 * t + ks) * 64 + lane] = v;
      }
  }
  for (int i = threadIdx.x; i < 2 * MH; i += blockDim.x) cv[i] = P[i < MH ? OFF_B1 + i : OFF_B2 + i - MH];
  f.cv = cv;
  f.a2l = a2l;
  f.b3 = P[OFF_B3];
  __syncthreads();
}

// ReLU on the bit pattern: a float with the sign bit clear compares as a
// non-negative int32 in the same order, one with it set as a negative one,
// so max(bits, 0) is max(x, +0) in one integer instruction.
__device__ __forceinline__ float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// One K-step of the next layer's B operand from two 16-unit row tiles of
// this layer's accumulators (lane: units 16 t + 4 kq + j of its symbol, t =
// 2 ks, 2 ks + 1): each pair rounded to BF16, then ReLU as a packed 16-bit
// integer max with 0.
__device__ __forceinline__ void mlp_handover(const rx_f32x4 &da, const rx_f32x4 &db, MNT::vec &out) {
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int jp = 0; jp < 4; jp++) {
    const rx_f32x4 &d = jp < 2 ? da : db;
    const int j = (2 * jp) % 4;
    bf16x2 pr = __builtin_convertvector((f32x2){d[j], d[j + 1]}, bf16x2);
    s16x2 bits = __builtin_bit_cast(s16x2, pr);
    bits = __builtin_elementwise_max(bits, (s16x2){0, 0});
    pr = __builtin_bit_cast(bf16x2, bits);
    out[2 * jp] = pr[0];
    out[2 * jp + 1] = pr[1];
  }
}

// NT tiles of 16 symbols at once (their dependent MFMA -> VALU chains
// interleave, which one tile's chain alone leaves the SIMD idle waiting
// on); bx[i] = this lane's B fragment of layer 1 for tile i (window samples
// 8 kq .. 8 kq + 7 of symbol `row`).  Lanes with kq == 0 return in y[i]
// the output of symbol `row` of tile i (the other lanes hold b3).  Registers
// and LDS reads of the bias vectors only; no cross-lane traffic.
// A2L: the W2 fragments from LDS (f.a2l) at lane index a2i, read per call.
template <int NT, bool A2L = false>
__device__ __forceinline__ void mlp_tiles(const MlpFrag &f, const MNT::vec (&bx)[NT], int kq, float (&y)[NT],
                                          int a2i = 0) {
  const float4 *cv4 = reinterpret_cast<const float4 *>(f.cv) + kq;   // units 16 t + 4 kq .. + 3
  rx_f32x4 d1[NT][4];
#pragma unroll
  for (int t = 0; t < 4; t++) {
    const float4 b = cv4[4 * t];
#pragma unroll
    for (int i = 0; i < NT; i++) d1[i][t] = MNT::mfma(f.a1[t], bx[i], rx_f32x4{b.x, b.y, b.z, b.w});
  }
  // layer-1 activations: round pairs to BF16, then ReLU as a packed 16-bit
  // integer max with 0 (a BF16 with the sign bit set is a negative int16;
  // rounding and ReLU commute); the same hand-over takes layer 2's outputs
  // to layer 3
  MNT::vec bh[NT][2];
#pragma unroll
  for (int i = 0; i < NT; i++)
#pragma unroll
    for (int ks = 0; ks < 2; ks++) mlp_handover(d1[i][2 * ks], d1[i][2 * ks + 1], bh[i][ks]);
  // layer 2, two 16-unit row tiles at a time (one K-step of layer 3's B)
  MNT::vec bh2[NT][2];
#pragma unroll
  for (int ks = 0; ks < 2; ks++) {
    rx_f32x4 d[NT][2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int t = 2 * ks + h;
      const float4 b = cv4[16 + 4 * t];
      const MNT::vec w20 = A2L ? f.a2l[(2 * t) * 64 + a2i] : f.a2[t][0];
      const MNT::vec w21 = A2L ? f.a2l[(2 * t + 1) * 64 + a2i] : f.a2[t][1];
#pragma unroll
      for (int i = 0; i < NT; i++) d[i][h] = MNT::mfma(w20, bh[i][0], rx_f32x4{b.x, b.y, b.z, b.w});
#pragma unroll
      for (int i = 0; i < NT; i++) d[i][h] = MNT::mfma(w21, bh[i][1], d[i][h]);
    }
#pragma unroll
    for (int i = 0; i < NT; i++) mlp_handover(d[i][0], d[i][1], bh2[i][ks]);
  }
  // layer 3: lane l < 16 gets y of symbol l in element 0
#pragma unroll
  for (int i = 0; i < NT; i++) {
    rx_f32x4 o = MNT::mfma(f.a3[0], bh2[i][0], rx_f32x4{0.0f, 0.0f, 0.0f, 0.0f});
    o = MNT::mfma(f.a3[1], bh2[i][1], o);
    y[i] = o[0] + f.b3;
  }
}

// Five wavefronts per SIMD (at most 102 VGPRs; it needs 88): the loop waits
// on its LDS and MFMA results, and a fifth wavefront hides more of that.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void mlp_infer(RxLaunch L) {
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  if (!J.mlp) return;
  const int64_t n = L.n[jb], nsym = n / 2;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar tile bookkeeping
  const int row = lane & 15, kq = lane >> 4;
  const int s = J.sc->lag;
  const auto xr = gptr(J.xr);
  __shared__ __attribute__((aligned(16))) float cv[2 * MH];
  // the W2 fragments in LDS, read per tile pair: held in registers they kept
  // the kernel at three wavefronts per SIMD
  __shared__ MNT::vec a2l[8 * 64];
  MlpFrag f;
  mlp_load_frag(J.mlp, row, kq, cv, f, a2l);
  const int64_t tile0 = ((int64_t)blockIdx.x * 4 + wv) * MLP_INFER_TPW;
  const int64_t ntl = (nsym - 16 * tile0 + 15) / 16;
  const int nt = ntl < MLP_INFER_TPW ? (int)ntl : MLP_INFER_TPW;   // this wave's tiles (none if <= 0)
  // Window sample 8 kq + j of symbol k0 + row is x[2 (k0 + row + s) - 15 + 8 kq + j]
  // = x[w0 + 32 tt + lo + j] with w0 = 2 (16 tile0 + s) - 15 (the wave's first
  // window) and lo = 2 row + 8 kq < 64.  A step (two tiles, tt and tt + 1)
  // reads samples w0 + 32 tt + [0, 94): the wave loads 128 of them (two per
  // lane, one read per sample instead of one per window it falls in),
  // rounds each pair to BF16 once and parks the pairs in its own LDS
  // staging area, from which every lane reads its B fragments.  Copy 0
  // holds pair p (samples 2p, 2p + 1) at dword p, copy 1 at dword p - 1, so
  // a lane's four dwords p0 = row + 4 kq + 16 i .. p0 + 3 start 8-byte
  // aligned in copy row & 1.  Two areas alternate by step; the next step's
  // samples load while a step runs.  Samples outside the buffer read as 0
  // (only near its ends: a wave-uniform test picks the guarded path).
  const int64_t w0 = 2 * (16 * tile0 + s) - 15;
  __shared__ __attribute__((aligned(16))) uint32_t xs[4][2][2][64];   // [wave][area][copy][dword]
  uint32_t(*const xw)[2][64] = xs[wv];
  auto load_x = [&](int tt, float (&xv)[2]) {
    const int64_t t0 = w0 + 32 * (int64_t)tt;
    if (t0 >= 0 && t0 + 127 < n) {
      const auto tp = xr + t0;
      xv[0] = tp[2 * lane];
      xv[1] = tp[2 * lane + 1];
    } else {
#pragma unroll
      for (int e = 0; e < 2; e++) {
        const int64_t q = t0 + 2 * lane + e;
        xv[e] = (q >= 0 && q < n) ? xr[q] : 0.0f;
      }
    }
  };
  auto stage = [&](int area, const float (&xv)[2]) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const uint32_t pr = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){xv[0], xv[1]}, bf16x2));
    xw[area][0][lane] = pr;
    xw[area][1][(lane + 63) & 63] = pr;   // lane 0's copy-1 slot (dword 63) is never read
  };
  const int rpar = row & 1, p0 = row - rpar + 4 * kq;   // this lane's first dword, even
  // two tiles per step (the second past the wave's last tile is computed on
  // in-buffer samples and not stored); the loop takes two steps per
  // iteration, so the staging area of each is a constant
  auto step = [&](int tt, int area, float (&xv)[2]) {
    MNT::vec bx[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
      const uint2 *src = reinterpret_cast<const uint2 *>(&xw[area][rpar][p0 + 16 * i]);
      const uint2 u = src[0], v = src[1];
      bx[i] = __builtin_bit_cast(MNT::vec, (uint4){u.x, u.y, v.x, v.y});
    }
    load_x(tt + 2, xv);   // the next step's samples, in flight during this one
    float y[2];
    // the fragment index is re-formed each step, so the reads are not
    // hoisted out of the loop into registers
    int a2i = lane;
    asm volatile("" : "+v"(a2i));
    mlp_tiles<2, true>(f, bx, kq, y, a2i);
#pragma unroll
    for (int i = 0; i < 2; i++) {
      const int64_t k = (tile0 + tt + i) * 16 + row;
      if (kq == 0 && tt + i < nt && k < nsym) gptr(reinterpret_cast<float *>(J.soft))[k] = y[i];   // PAM: real soft symbols
    }
    // the other area takes the next step's pairs; a wavefront's LDS
    // accesses run in program order, so only the compiler needs the fence
    stage(area ^ 1, xv);
    wave_sync();
  };
  {
    float xv[2];
    load_x(0, xv);
    stage(0, xv);
    wave_sync();
  }
  float xv[2];
  for (int tt = 0; tt < nt; tt += 4) {
    step(tt, 0, xv);
    if (tt + 2 >= nt) break;
    step(tt + 2, 1, xv);
  }
}

// The same inference on given rows X[n][32] (column 31 ignored) -> Y[n].
__global__ __launch_bounds__(256) void mlp_infer_rows(const float *__restrict__ P, const float *__restrict__ X,
                                                      int64_t nrows, float *__restrict__ Y) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = lane & 15, kq = lane >> 4;
  __shared__ __attribute__((aligned(16))) float cv[2 * MH];
  MlpFrag f;
  mlp_load_frag(P, row, kq, cv, f);
  const int64_t tile0 = ((int64_t)blockIdx.x * 4 + wv) * TILES_PER_WAVE;
  for (int tt = 0; tt < TILES_PER_WAVE; tt++) {
    const int64_t r = (tile0 + tt) * 16 + row;
    if ((tile0 + tt) * 16 >= nrows) break;
    MNT::vec bx[1];
#pragma unroll
    for (int j = 0; j < 8; j++) bx[0][j] = MNT::cvt((8 * kq + j < MI && r < nrows) ? X[r * 32 + 8 * kq + j] : 0.0f);
    float y[1];
    mlp_tiles<1>(f, bx, kq, y);
    if (kq == 0 && r < nrows) Y[r] = y[0];
  }
}

// LMS stays the fallback and the judge: on the known prefix symbols
// [64, prefix) count the MLP's decision errors and those of the FFE with the
// trained prefix taps w0; the block DD-LMS runs (and overwrites the MLP's
// soft symbols) when the MLP makes more errors.
__global__ __launch_bounds__(256) void mlp_judge(RxLaunch L) {
  __shared__ double red[4];
  const int jb = blockIdx.y;
  const RxJob J = *L.job[jb];
  const int64_t n = L.n[jb];
  const int K = J.ffe_taps, C = (K - 1) / 2, P = J.prefix, m = J.m_axis;
  const int s = J.sc->lag;
  double em = 0.0, el = 0.0;
  for (int k = RX_GUARD + threadIdx.x; k < P; k += 256) {
    const float a = ref_symbol(J, k).x;
    em += decide_level(reinterpret_cast<const float *>(J.soft)[k], m) != a;
    float z = 0.0f;
    for (int i = 0; i < K; i++) {
      const int64_t j = 2 * ((int64_t)k + s) + C - i;
      z = fmaf(J.sc->w0[i].x, (j >= 0 && j < n) ? J.xr[j] : 0.0f, z);
    }
    el += decide_level(z, m) != a;
  }
  em = block_sum(em, red);
  el = block_sum(el, red);
  if (threadIdx.x == 0) J.sc->fallback = em > el ? 1 : 0;
}

// ---- host-side launchers ---------------------------------------------------
void rx_launch_mlp_stage(int stage, const RxLaunch &L, int64_t maxn, hipStream_t s) {
  const unsigned cnt = (unsigned)L.count;
  const int64_t nsym = maxn / 2;
  if (stage == ST_MLP_INFER) {
    const int64_t tiles = (nsym + 15) / 16;
    const int64_t wgs = (tiles + 4 * MLP_INFER_TPW - 1) / (4 * MLP_INFER_TPW);
    hipLaunchKernelGGL(mlp_infer, dim3((unsigned)wgs, cnt), dim3(256), 0, s, L);
  } else if (stage == ST_MLP_JUDGE) {
    hipLaunchKernelGGL(mlp_judge, dim3(1, cnt), dim3(256), 0, s, L);
  }
}

void rx_mlp_windows(const RxLaunch &L, float *X, float *T, int64_t row0, hipStream_t s) {
  const int64_t nsym = L.n[0] / 2;
  const int64_t rows = nsym - 2 * RX_GUARD;
  hipLaunchKernelGGL(mlp_windows, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, L, X, T, row0);
}

int rx_mlp_params(void) { return MP; }

void rx_mlp_infer_rows(const float *P, const float *X, int64_t n, float *Y, hipStream_t s) {
  const int64_t tiles = (n + 15) / 16;
  const int64_t wgs = (tiles + 4 * TILES_PER_WAVE - 1) / (4 * TILES_PER_WAVE);
  hipLaunchKernelGGL(mlp_infer_rows, dim3((unsigned)wgs), dim3(256), 0, s, P, X, n, Y);
}

void rx_mlp_step(const float *X, const float *T, int64_t ntrain, int64_t i0, int batch, int64_t mult, float *p,
                 float *m, float *v, float *part, double *loss_part, float *grad, int adam, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t s) {
  const int nwg = (batch + SPW - 1) / SPW;
  hipLaunchKernelGGL(mlp_grad_partial, dim3(nwg), dim3(256), 0, s, p, X, T, ntrain, i0, batch, mult, part,
                     loss_part);
  hipLaunchKernelGGL(mlp_reduce_adam, dim3((MP + 255) / 256), dim3(256), 0, s, p, m, v, part, nwg, grad, adam, lr,
                     b1, b2, eps, c1, c2);
}

// ---- the gradient's partials in a static device array ---------------------
// For callers that cannot allocate: RX_MLP_STATIC_ROWS rows at most, i.e.
// RX_MLP_STATIC_ROWS / SPW workgroup partials of MP floats, then as many
// FP64 loss partials.  Every workgroup writes all of its partial (nothing
// has to start at zero); each GPU holds one copy until the process ends.
#define RX_STATIC_PARTS (RX_MLP_STATIC_ROWS / SPW)
static_assert((RX_STATIC_PARTS * MP) % 2 == 0, "the FP64 loss partials start 8-byte aligned");
static __device__ __align__(256) float scratch[RX_STATIC_PARTS * MP + 2 * RX_STATIC_PARTS];

// The array's device address on the current device, resolved once per
// device (in host code the array's name is no device address).
int rx_mlp_scratch_resolve(void **out) {
  static std::mutex mu;
  static std::map<int, void *> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return e != hipSuccess ? (int)e : (int)hipErrorInvalidSymbol;
    it = addr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return 0;
}

int rx_mlp_scratch_parts(void) { return RX_STATIC_PARTS; }

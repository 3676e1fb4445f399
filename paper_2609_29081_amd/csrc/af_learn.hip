// af_learn.hip -- the learned blend coefficient of the 2D cell-average fluxes
// on gfx950: face features, inference of the 40-64-64-1 network on the MFMA
// units, and the network's training (loss gradient and Adam).
//
// The network proposes, per face, the coefficient that blends the low- and
// high-order cell-average fluxes in place of the smoothness blend theta^s of
// Sec. 3.2; the density/pressure limiter of Sec. 3.3 then clamps it as it
// clamps theta^s (the coefficient used is theta_nn theta^rho theta^p, never
// above theta_nn nor the admissible bound), and the face flux stays
// single-valued (conservative).
//
// Features of a face (a, b its minus and plus cells): in the face's frame
// (normal n along its axis, tangent t along the other) the 4 x 3 block of
// cell averages at normal offsets -2, -1 (a), +1 (b), +2 and tangential
// offsets -1, 0, +1, ghost cells being boundary images.  With face values
// rho_f = (rho_a + rho_b)/2, p_f, u_nf, u_tf likewise and
// c_f = sqrt(gamma p_f / rho_f): for s = -1, 0, +1 and m = -2, -1, +1, +2 the
// triple [ln(p / p_f), (u_n - u_nf) / c_f, (u_t - u_tf) / c_f], then
// ln(rho / rho_f) for m = -2, -1, +1, +2 at s = 0 (40 values).
//
// Network: h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), z = w3.h2 + b3,
// theta_nn = min(max(z, 0), 1); parameters as one FP32 vector
// [W1 (64 x 40, row-major), b1, W2 (64 x 64), b2, w3, b3].  Inference keeps
// W1, W2, w3 and the layer inputs x, h1 in bfloat16 (round to nearest even)
// and accumulates in FP32 (MFMA 32x32x16 bf16); training runs in FP32.
#include "af_device.hpp"
#include "af_internal.hpp"
#include "af_lattice.hpp"

using namespace afd;

namespace {

constexpr int NIN = afi::kMlpIn, NH = afi::kMlpHidden;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH;
static_assert(OFF_B3 + 1 == afi::kMlpParams, "parameter layout");

// packed inference weights: bfloat16 W1 [64][40], W2 [64][64], w3 [64], then
// FP32 b1 [64], b2 [64], b3
constexpr int PK_W1 = 0, PK_W2 = PK_W1 + 2 * NH * NIN, PK_W3 = PK_W2 + 2 * NH * NH,
              PK_B1 = PK_W3 + 2 * NH, PK_B2 = PK_B1 + 4 * NH, PK_B3 = PK_B2 + 4 * NH;
static_assert(PK_B3 + 4 <= (int)afi::kMlpPackedBytes, "packed weights");

// round to nearest even (one hardware conversion on gfx950)
__device__ __forceinline__ unsigned short to_bf16(float x) {
  return __builtin_bit_cast(unsigned short, (__bf16)x);
}
__device__ __forceinline__ float from_bf16(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}

// face f -> direction d, face (i, j); x-faces [n2][n1+1] first
__device__ __forceinline__ void face_of(const G2& g, long f, int& d, int& i, int& j) {
  const long nfx = (long)g.n2 * (g.n1 + 1);
  if (f < nfx) {
    d = 0;
    j = (int)(f / (g.n1 + 1));
    i = (int)(f % (g.n1 + 1));
  } else {
    d = 1;
    const long r = f - nfx;
    j = (int)(r / g.n1);
    i = (int)(r % g.n1);
  }
}

// (rho, u, v, p) as FP32 from a cell average (FP64 arithmetic)
__device__ __forceinline__ void prims_of(double gm1, const double* V, float* P) {
  const double ir = 1.0 / V[0], u = V[1] * ir, v = V[2] * ir;
  P[0] = float(V[0]);
  P[1] = float(u);
  P[2] = float(v);
  P[3] = float(gm1 * (V[3] - 0.5 * V[0] * (u * u + v * v)));
}

// (rho, u, v, p) of the cell average of cell (ci, cj), ci in [-2, n1+1]
__device__ __forceinline__ void cell_prims(const G2& g, double gm1, const double* U, int ci, int cj,
                                           float* P) {
  double V[4];
  raw_value(g, U, 2 * ci + 1, 2 * cj + 1, V);
  prims_of(gm1, V, P);
}

__device__ __forceinline__ float pos_or_tiny(float v) { return v > 1e-30f ? v : 1e-30f; }

// features of face (d, i, j) from the primitives of its stencil cells:
// cell(s, q, P) fills the (rho, u, v, p) of tangential offset s-1 and normal
// offset q in (-2, -1, +1, +2).  Half h of the features (h = 0, 1; -1 for
// all) is the triples of stencil cells 6h .. 6h+5 (cell 4s+q) and the
// density ratios of q = 2h, 2h+1; put(n, value) receives feature n.
template <typename CellFn, typename PutFn>
__device__ __forceinline__ void features_of(int d, float gam, CellFn cell, PutFn put,
                                            int h = -1) {
  const int c0 = h < 0 ? 0 : 6 * h, c1 = h < 0 ? 12 : 6 * h + 6;
  const int q0 = h < 0 ? 0 : 2 * h, q1 = h < 0 ? 4 : 2 * h + 2;
  // face values from the two cells that adjoin the face
  float A[4], B[4];
  cell(1, 1, A);
  cell(1, 2, B);
  const float rf = 0.5f * (A[0] + B[0]), pf = 0.5f * (A[3] + B[3]);
  const float unf = 0.5f * (d == 0 ? A[1] + B[1] : A[2] + B[2]);
  const float utf = 0.5f * (d == 0 ? A[2] + B[2] : A[1] + B[1]);
  const float icf = 1.0f / sqrtf(gam * pos_or_tiny(pf) / pos_or_tiny(rf));
  const float ipf = 1.0f / pos_or_tiny(pf), irf = 1.0f / pos_or_tiny(rf);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    if (c < c0 || c >= c1) continue;
    float P[4];
    cell(c / 4, c % 4, P);
    const float un = d == 0 ? P[1] : P[2], ut = d == 0 ? P[2] : P[1];
    put(3 * c, __logf(pos_or_tiny(P[3]) * ipf));
    put(3 * c + 1, (un - unf) * icf);
    put(3 * c + 2, (ut - utf) * icf);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < q0 || q >= q1) continue;
    float P[4];
    cell(1, q, P);
    put(36 + q, __logf(pos_or_tiny(P[0]) * irf));
  }
}

// tanh from the exponential: 1 - 2 / (1 + e^{2x}), with the hardware
// exponential and reciprocal (the result feeds bfloat16 operands; its error
// is far below their rounding)
__device__ __forceinline__ float tanh_fast(float x) {
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * x));
}

// stencil cell (ci, cj) of face (d, i, j) at tangential offset s-1, normal
// offset index q
__device__ __forceinline__ void stencil_cell(int d, int i, int j, int s, int q, int& ci, int& cj) {
  const int m = q - 2;  // -2, -1, 0, +1 relative to cell b
  if (d == 0) {
    ci = i + m;
    cj = j + s - 1;
  } else {
    ci = i + s - 1;
    cj = j + m;
  }
}

// ---------------------------------------------------------------------------
// features of every face (training data), one thread per face
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_features(G2 g, double gm1, float gam,
                                                  const double* __restrict__ U,
                                                  float* __restrict__ out, long nf) {
  for (long f = blockIdx.x * (long)blockDim.x + threadIdx.x; f < nf;
       f += (long)gridDim.x * blockDim.x) {
    int d, i, j;
    face_of(g, f, d, i, j);
    features_of(d, gam,
                [&](int s, int q, float* P) {
                  int ci, cj;
                  stencil_cell(d, i, j, s, q, ci, cj);
                  cell_prims(g, gm1, U, ci, cj, P);
                },
                [&](int n, float v) { out[f * NIN + n] = v; });
  }
}

// ---------------------------------------------------------------------------
// inference.  A workgroup (four wave64s) takes 128 consecutive faces of
// each of eight rows of one direction: it stages the primitives of their
// stencil cells in LDS once (ten rows of cells for eight rows of x-faces,
// eleven for y-faces, where one face row at a time needed three or four),
// and for each face row writes the features as bfloat16 rows; each wave
// then runs the network on 32 faces with MFMA 32x32x16 bf16 in the
// transposed form H^T = W X^T: the weights are the A operand (units x
// inputs, in registers), the faces the columns.  A 32 x 32 accumulator holds
// in lane (face c, half h) the rows (units) 8 (r/4) + 4 h + r%4 of column c,
// r = 0..15, and the B operand of the next layer needs in that lane the
// inputs 16 kb + 8 h + e, e = 0..7, of the same face: registers 8q .. 8q+7
// of the accumulator of unit block nb are exactly that for kb = 2 nb + q,
// once the hidden units are numbered in that (virtual) order, which is how
// layer 2's weights are stored.  So hidden values never leave the
// registers, and the output layer's sum over units ends with one exchange
// between the two halves of the wave.
// ---------------------------------------------------------------------------
constexpr int IB = 128;                 // faces per row of a block
constexpr int RB = 8;                   // face rows per block, at most
constexpr int KIN = 48;                 // inputs padded to three K steps of 16
constexpr int FROW = KIN + 8;           // feature row (bf16; 16-byte aligned)
constexpr int CW = IB + 4;              // stencil cells per row

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct InferShared {
  float cell[4][RB + 3][CW];            // [component][row][column]
  unsigned short feat[IB * FROW];
  float b1[NH], b2[NH], w3[NH];         // biases, and the output weights (bf16 values)
  // layer 2's A operands, per lane (in LDS rather than registers: with them
  // in registers the kernel holds 188 VGPRs, two waves per SIMD, and ran 18 %
  // slower at 2048 x 1024)
  bf16x8 a2[2][4][64];
};

__device__ __forceinline__ bf16x8 bf16x8_of(const unsigned short* p, int n) {
  bf16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = __builtin_bit_cast(__bf16, e < n ? p[e] : (unsigned short)0);
  return v;
}

// unit of layer-2 input (virtual) index k, for the half h of the lanes that
// holds it: kb = k / 16 = 2 nb + q, e = k % 8 = 4 a + i (see above)
__device__ __forceinline__ int hidden_unit(int kb, int h, int e) {
  const int nb = kb >> 1, q = kb & 1, a = e >> 2, i = e & 3;
  return 32 * nb + 8 * (2 * q + a) + 4 * h + i;
}

// at least three waves per SIMD (at most 168 VGPRs)
__global__ void __launch_bounds__(256, 3) k_infer(G2 g, double gm1, float gam,
                                               const double* __restrict__ U,
                                               const unsigned char* __restrict__ pk,
                                               float* __restrict__ theta, int nsegx, int nsegy,
                                               int rb, long nblocks) {
  __shared__ InferShared S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, c32 = lane & 31;
  const unsigned short* W1 = (const unsigned short*)(pk + PK_W1);
  const unsigned short* W2 = (const unsigned short*)(pk + PK_W2);
  const unsigned short* w3 = (const unsigned short*)(pk + PK_W3);
  const float* b1 = (const float*)(pk + PK_B1);
  const float* b2 = (const float*)(pk + PK_B2);
  const float b3 = *(const float*)(pk + PK_B3);
  // A operands: lane (m = c32, h) holds row 32 nb + m, inputs 16 kb + 8 h + e
  // (layer 2's written to LDS by the first wave, read after the first barrier)
  bf16x8 A1[2][3];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
    for (int kb = 0; kb < 3; ++kb) {
      const int k0 = 16 * kb + 8 * h;
      A1[nb][kb] = bf16x8_of(W1 + (32 * nb + c32) * NIN + (k0 < NIN ? k0 : 0),
                             k0 < NIN ? NIN - k0 : 0);
    }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        v[e] = __builtin_bit_cast(__bf16, W2[(32 * nb + c32) * NH + hidden_unit(kb, h, e)]);
      if (wave == 0) S.a2[nb][kb][lane] = v;
    }
  }
  for (int e = tid; e < NH; e += 256) {
    S.b1[e] = b1[e];
    S.b2[e] = b2[e];
    S.w3[e] = from_bf16(w3[e]);
  }
  const long nfx = (long)g.n2 * (g.n1 + 1);
  const long ngx = (g.n2 + rb - 1) / rb;  // row groups of the x-faces
  const long nbx = ngx * nsegx;
  // block blk: direction, first row and row count, first face along the
  // rows, face count per row, and its stencil cells: x-faces need columns
  // i0-2 .. i0+cnt and rows row0-1 .. row0+nr, y-faces columns i0-1 ..
  // i0+cnt and rows row0-2 .. row0+nr-1
  struct Blk {
    int d, row0, nr, i0, cnt, ncol, nrow, c0, r0;
  };
  auto block_of = [&](long blk) {
    Blk b;
    if (blk < nbx) {
      b.d = 0;
      b.row0 = (int)(blk / nsegx) * rb;
      b.nr = min(rb, g.n2 - b.row0);
      b.i0 = (int)(blk % nsegx) * IB;
      b.cnt = min(IB, g.n1 + 1 - b.i0);
    } else {
      b.d = 1;
      const long r = blk - nbx;
      b.row0 = (int)(r / nsegy) * rb;
      b.nr = min(rb, g.n2 + 1 - b.row0);
      b.i0 = (int)(r % nsegy) * IB;
      b.cnt = min(IB, g.n1 - b.i0);
    }
    b.ncol = b.d == 0 ? b.cnt + 3 : b.cnt + 2;
    b.nrow = (b.d == 0 ? 2 : 3) + b.nr;
    b.c0 = b.d == 0 ? b.i0 - 2 : b.i0 - 1;
    b.r0 = b.d == 0 ? b.row0 - 1 : b.row0 - 2;
    return b;
  };
  // the FP64 averages of a block's stencil cells, up to (RB + 3) x 130 cells,
  // loaded at the start of the block (held one block ahead, they took more
  // registers than three workgroups per CU leave; the other workgroups on the
  // CU hide the wait)
  constexpr int CPT = ((RB + 3) * (IB + 2) + 255) / 256;
  static_assert((RB + 2) * (IB + 3) <= CPT * 256 && (RB + 3) * (IB + 2) <= CPT * 256,
                "cells per thread");
  double pre[CPT][4];
  auto fetch = [&](const Blk& b) {
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      const int e = tid + 256 * r;
      if (e < b.ncol * b.nrow) raw_value(g, U, 2 * (b.c0 + e % b.ncol) + 1, 2 * (b.r0 + e / b.ncol) + 1, pre[r]);
    }
  };
  long blk = blockIdx.x;
  for (; blk < nblocks; blk += gridDim.x) {
    const Blk B = block_of(blk);
    fetch(B);
    const int d = B.d, i0 = B.i0, cnt = B.cnt, c0 = B.c0, r0 = B.r0;
    __syncthreads();  // the previous block is done with the cell and feature arrays
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
      const int e = tid + 256 * r;
      if (e < B.ncol * B.nrow) {
        float P[4];
        prims_of(gm1, pre[r], P);
#pragma unroll
        for (int k = 0; k < 4; ++k) S.cell[k][e / B.ncol][e % B.ncol] = P[k];
      }
    }
    for (int rr = 0; rr < B.nr; ++rr) {
      const int row = B.row0 + rr;
      __syncthreads();  // the cells are in; the previous row is done with the features
      {
        // two threads per face, one half of its features each; inputs 40..47
        // are zero
        const int fl = tid & (IB - 1), half = tid / IB;
        unsigned short* fo = S.feat + fl * FROW;
        if (fl < cnt) {
          const int i = i0 + fl;
          features_of(d, gam,
                      [&](int s, int q, float* P) {
                        int ci, cj;
                        stencil_cell(d, i, row, s, q, ci, cj);
#pragma unroll
                        for (int k = 0; k < 4; ++k) P[k] = S.cell[k][cj - r0][ci - c0];
                      },
                      [&](int n, float v) { fo[n] = to_bf16(v); }, half);
        } else {
          for (int n = half; n < NIN; n += 2) fo[n] = 0;
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) fo[NIN + 4 * half + n] = 0;
      }
      __syncthreads();
      // the wave's 32 faces: lane (c32, h) works on face 32 wave + c32
      const unsigned short* fa = S.feat + (32 * wave + c32) * FROW;
      f32x16 acc[2];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[nb][r] = 0.0f;
#pragma unroll
      for (int kb = 0; kb < 3; ++kb) {
        const bf16x8 x = *reinterpret_cast<const bf16x8*>(fa + 16 * kb + 8 * h);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1[nb][kb], x, acc[nb], 0, 0, 0);
      }
      // h1 = tanh(W1 x + b1) in bfloat16: layer 2's B operand, kb = 2 nb + q
      bf16x8 hb[4];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float4 bias = *reinterpret_cast<const float4*>(&S.b1[32 * nb + 8 * j + 4 * h]);
          const float bj[4] = {bias.x, bias.y, bias.z, bias.w};
#pragma unroll
          for (int i = 0; i < 4; ++i)
            hb[2 * nb + (j >> 1)][4 * (j & 1) + i] = (__bf16)tanh_fast(acc[nb][4 * j + i] + bj[i]);
        }
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[nb][r] = 0.0f;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(S.a2[nb][kb][lane], hb[kb], acc[nb], 0, 0, 0);
      // z = w3 . tanh(W2 h1 + b2) + b3: this lane's 32 units of its face, then
      // the other half's 32 from the lane 32 away
      float z = 0.0f;
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = 32 * nb + 8 * j + 4 * h;
          const float4 bias = *reinterpret_cast<const float4*>(&S.b2[u]);
          const float4 ow = *reinterpret_cast<const float4*>(&S.w3[u]);
          z += ow.x * tanh_fast(acc[nb][4 * j] + bias.x);
          z += ow.y * tanh_fast(acc[nb][4 * j + 1] + bias.y);
          z += ow.z * tanh_fast(acc[nb][4 * j + 2] + bias.z);
          z += ow.w * tanh_fast(acc[nb][4 * j + 3] + bias.w);
        }
      z += __shfl_xor(z, 32, 64);
      const int m = 32 * wave + c32;
      if (h == 0 && m < cnt) {
        const long f = (d == 0 ? 0 : nfx) + (long)row * (d == 0 ? g.n1 + 1 : g.n1) + i0 + m;
        theta[f] = fminf(fmaxf(z + b3, 0.0f), 1.0f);
      }
    }
  }
}

__global__ void k_pack(const float* __restrict__ p, unsigned char* __restrict__ pk) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < NH * NIN) ((unsigned short*)(pk + PK_W1))[t] = to_bf16(p[OFF_W1 + t]);
  if (t < NH * NH) ((unsigned short*)(pk + PK_W2))[t] = to_bf16(p[OFF_W2 + t]);
  if (t < NH) {
    ((unsigned short*)(pk + PK_W3))[t] = to_bf16(p[OFF_W3 + t]);
    ((float*)(pk + PK_B1))[t] = p[OFF_B1 + t];
    ((float*)(pk + PK_B2))[t] = p[OFF_B2 + t];
  }
  if (t == 0) *(float*)(pk + PK_B3) = p[OFF_B3];
}

// ---------------------------------------------------------------------------
// training: gradient of the mean squared error over n samples, FP32.  Each
// workgroup takes chunks of 64 samples, runs forward and backward through
// LDS and accumulates its share of the gradient in registers; partial
// gradients are then summed in a fixed order (deterministic).
// ---------------------------------------------------------------------------
constexpr int GC = 64;          // samples per chunk
constexpr int GT = 256;         // threads per workgroup
constexpr int kGradBlocks = 128;

struct GradShared {
  float W1[NH * NIN], W2[NH * NH], w3[NH], b1[NH], b2[NH];
  float X[GC * NIN], H1[GC * NH], H2[GC * NH], A[GC * NH], dz[GC], red[GT];
};

__global__ void __launch_bounds__(GT) k_grad(const float* __restrict__ X,
                                             const float* __restrict__ y, long n,
                                             const float* __restrict__ p,
                                             float* __restrict__ part, float inv_n) {
  __shared__ GradShared S;
  const int t = threadIdx.x;
  for (int e = t; e < NH * NIN; e += GT) S.W1[e] = p[OFF_W1 + e];
  for (int e = t; e < NH * NH; e += GT) S.W2[e] = p[OFF_W2 + e];
  if (t < NH) {
    S.w3[t] = p[OFF_W3 + t];
    S.b1[t] = p[OFF_B1 + t];
    S.b2[t] = p[OFF_B2 + t];
  }
  const float b3 = p[OFF_B3];
  float gW1[10], gW2[16], gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, loss = 0.f;
#pragma unroll
  for (int r = 0; r < 10; ++r) gW1[r] = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) gW2[r] = 0.f;
  const int nu = t & 63, mg = t >> 6;  // unit and sample group of this thread
  const long nchunk = (n + GC - 1) / GC;
  for (long c = blockIdx.x; c < nchunk; c += gridDim.x) {
    const long base = c * GC;
    __syncthreads();
    for (int e = t; e < GC * NIN; e += GT) {
      const long row = base + e / NIN;
      S.X[e] = row < n ? X[row * NIN + e % NIN] : 0.f;
    }
    __syncthreads();
    // layer 1
#pragma unroll 1
    for (int r = 0; r < 16; ++r) {
      const int m = 16 * mg + r;
      float a = S.b1[nu];
#pragma unroll 8
      for (int k = 0; k < NIN; ++k) a += S.W1[nu * NIN + k] * S.X[m * NIN + k];
      S.H1[m * NH + nu] = tanhf(a);
    }
    __syncthreads();
    // layer 2
#pragma unroll 1
    for (int r = 0; r < 16; ++r) {
      const int m = 16 * mg + r;
      float a = S.b2[nu];
#pragma unroll 8
      for (int k = 0; k < NH; ++k) a += S.W2[nu * NH + k] * S.H1[m * NH + k];
      S.H2[m * NH + nu] = tanhf(a);
    }
    __syncthreads();
    // output, residual, dL/dz
    if (t < GC) {
      float z = b3;
      for (int k = 0; k < NH; ++k) z += S.w3[k] * S.H2[t * NH + k];
      const bool valid = base + t < n;
      const float res = valid ? z - y[base + t] : 0.f;
      loss += res * res;
      S.dz[t] = 2.f * res * inv_n;
    }
    __syncthreads();
    // dL/d(layer-2 pre-activation)
#pragma unroll 1
    for (int r = 0; r < 16; ++r) {
      const int m = 16 * mg + r;
      const float h2 = S.H2[m * NH + nu];
      S.A[m * NH + nu] = S.dz[m] * S.w3[nu] * (1.f - h2 * h2);
    }
    __syncthreads();
    if (t < NH) {
      float s3 = 0.f, s2 = 0.f;
      for (int m = 0; m < GC; ++m) {
        s3 += S.dz[m] * S.H2[m * NH + t];
        s2 += S.A[m * NH + t];
      }
      gw3 += s3;
      gb2 += s2;
    }
    if (t == 0) {
      float s = 0.f;
#pragma unroll 8
      for (int m = 0; m < GC; ++m) s += S.dz[m];
      gb3 += s;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = t + GT * r, o = e / NH, k = e % NH;
      float s = 0.f;
#pragma unroll 8
      for (int m = 0; m < GC; ++m) s += S.A[m * NH + o] * S.H1[m * NH + k];
      gW2[r] += s;
    }
    // dL/d(layer-1 pre-activation), into H2 (no longer needed)
#pragma unroll 1
    for (int r = 0; r < 16; ++r) {
      const int m = 16 * mg + r;
      float s = 0.f;
#pragma unroll 8
      for (int o = 0; o < NH; ++o) s += S.A[m * NH + o] * S.W2[o * NH + nu];
      const float h1 = S.H1[m * NH + nu];
      S.H2[m * NH + nu] = s * (1.f - h1 * h1);
    }
    __syncthreads();
    if (t < NH) {
      float s1 = 0.f;
      for (int m = 0; m < GC; ++m) s1 += S.H2[m * NH + t];
      gb1 += s1;
    }
#pragma unroll
    for (int r = 0; r < 10; ++r) {
      const int e = t + GT * r, o = e / NIN, k = e % NIN;
      float s = 0.f;
#pragma unroll 8
      for (int m = 0; m < GC; ++m) s += S.H2[m * NH + o] * S.X[m * NIN + k];
      gW1[r] += s;
    }
  }
  // this workgroup's partial gradient and loss sum
  float* q = part + (long)blockIdx.x * (afi::kMlpParams + 1);
#pragma unroll
  for (int r = 0; r < 10; ++r) q[OFF_W1 + t + GT * r] = gW1[r];
#pragma unroll
  for (int r = 0; r < 16; ++r) q[OFF_W2 + t + GT * r] = gW2[r];
  if (t < NH) {
    q[OFF_B1 + t] = gb1;
    q[OFF_B2 + t] = gb2;
    q[OFF_W3 + t] = gw3;
  }
  if (t == 0) q[OFF_B3] = gb3;
  S.red[t] = t < GC ? loss : 0.f;
  __syncthreads();
  if (t == 0) {
    float s = 0.f;
    for (int k = 0; k < GC; ++k) s += S.red[k];
    q[afi::kMlpParams] = s;
  }
}

__global__ void k_grad_sum(const float* __restrict__ part, int nparts, float* __restrict__ grad,
                           float* __restrict__ loss, float inv_n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > afi::kMlpParams) return;
  float s = 0.f;
  for (int b = 0; b < nparts; ++b) s += part[(long)b * (afi::kMlpParams + 1) + e];
  if (e < afi::kMlpParams)
    grad[e] = s;
  else if (loss)
    *loss = s * inv_n;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= afi::kMlpParams) return;
  const float ge = g[e];
  const float me = 0.9f * m[e] + 0.1f * ge;
  const float ve = 0.999f * v[e] + 0.001f * ge * ge;
  m[e] = me;
  v[e] = ve;
  p[e] -= lr * (me * c1) / (sqrtf(ve * c2) + 1e-8f);
}

}  // namespace

namespace afi {

hipError_t blend_features(const Geo& geo, const Phys& ph, const double* U, float* feat,
                          hipStream_t s) {
  const G2 g = stage_geo(geo);
  const long nf = (long)g.n2 * (g.n1 + 1) + (long)(g.n2 + 1) * g.n1;
  long nb = (nf + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_features, dim3((unsigned)nb), dim3(256), 0, s, g, ph.gm1, float(ph.gam), U,
                     feat, nf);
  return hipGetLastError();
}

hipError_t mlp_pack(const float* params, void* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3((NH * NH + 255) / 256), dim3(256), 0, s, params,
                     (unsigned char*)packed);
  return hipGetLastError();
}

// persistent workgroups of the inference kernel: as many as are resident
static int infer_workgroups() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cache[dev] == 0) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_infer, 256, 0) != hipSuccess ||
        per <= 0)
      per = 1;
    cache[dev] = cus * per;
  }
  return cache[dev];
}

hipError_t blend_infer(const Geo& geo, const Phys& ph, const double* U, const void* packed,
                       float* theta, hipStream_t s, Timer* tm) {
  const G2 g = stage_geo(geo);
  const int nsegx = (g.n1 + 1 + IB - 1) / IB, nsegy = (g.n1 + IB - 1) / IB;
  const long nwg = infer_workgroups();
  // rows per block: the most (up to RB) that still leave every resident
  // workgroup two blocks, so that a small grid keeps the device busy
  auto blocks = [&](int rb) {
    return (long)((g.n2 + rb - 1) / rb) * nsegx + (long)((g.n2 + 1 + rb - 1) / rb) * nsegy;
  };
  int rb = RB;
  while (rb > 1 && blocks(rb) < 2 * nwg) rb /= 2;
  const long nblocks = blocks(rb);
  const long grid = nblocks < nwg ? nblocks : nwg;
  AFI_TIMED(tm, 8, s,
            hipLaunchKernelGGL(k_infer, dim3((unsigned)grid), dim3(256), 0, s, g, ph.gm1,
                               float(ph.gam), U, (const unsigned char*)packed, theta, nsegx,
                               nsegy, rb, nblocks));
  return hipGetLastError();
}

size_t mlp_grad_workspace(long n) {
  (void)n;
  return sizeof(float) * (size_t)kGradBlocks * (kMlpParams + 1);
}

hipError_t mlp_grad(const float* X, const float* y, long n, const float* params, float* grad,
                    float* loss, void* ws, hipStream_t s) {
  const long nchunk = (n + GC - 1) / GC;
  const int nb = (int)(nchunk < kGradBlocks ? nchunk : kGradBlocks);
  float* part = (float*)ws;
  const float inv_n = 1.0f / float(n);
  hipLaunchKernelGGL(k_grad, dim3(nb), dim3(GT), 0, s, X, y, n, params, part, inv_n);
  hipLaunchKernelGGL(k_grad_sum, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, s,
                     (const float*)part, nb, grad, loss, inv_n);
  return hipGetLastError();
}

hipError_t mlp_adam(float* params, const float* grad, float* m, float* v, long step, float lr,
                    hipStream_t s) {
  const double c1 = 1.0 / (1.0 - pow(0.9, (double)step));
  const double c2 = 1.0 / (1.0 - pow(0.999, (double)step));
  hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, params, grad, m, v,
                     lr, float(c1), float(c2));
  return hipGetLastError();
}

}  // namespace afi

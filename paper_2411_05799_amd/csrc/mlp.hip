// The surrogate network of the batched simulator: a plain MLP
// (n_in -> n_hidden x n_hidden_layers -> n_out, SiLU between layers) trained on
// transitions the simulator generates, with hand-written matrix-core kernels
// for gfx950.
//
// Every product is one kernel form, C[M x N] = A[M x K] * B[N x K]^T with both
// operands k-contiguous, so that each lane's MFMA fragment is one 16-byte load:
//   forward   Z_l  = H_{l-1} * W_l^T          (A = activations, B = W_l)
//   input     dH   = dZ_l * W_l               (A = dZ_l, B = W_l^T copy)
//   weights   dW_l = dZ_l^T * H_{l-1}         (A = dZ_l^T, B = H_{l-1}^T), split over K
// Epilogues therefore also write the transposed copies the next product reads.
// BF16 operands with FP32 accumulation (v_mfma_f32_16x16x32_bf16) and FP32
// master weights, or FP32 operands throughout (v_mfma_f32_16x16x4f32) for
// checking gradients tightly.  Dimensions are padded to multiples of 64 with
// zeros that stay zero under training (their gradients vanish identically).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "npx.h"
#include "npx_internal.h"
#include "npx_sur_internal.h"

using npx::fail;

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(NPX_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));            \
  } while (0)

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TILE = 64;     // block tile edge (rows and columns)
constexpr int KSTEP = 32;    // k consumed per MFMA round

// ---- MFMA operand traits --------------------------------------------------
// A 16x16 output block is accumulated from 16-row slices of A and B: lane l
// supplies row (l mod 16) and the k-slice 8*(l/16) .. +8 of both operands; the
// result lands as D[4*(l/16)+e][l mod 16], e = 0..3.
template <class T>
struct Mfma;

template <>
struct Mfma<__bf16> {
  using frag = bf16x8;
  static __device__ __forceinline__ frag load(const __bf16* p) {
    return *reinterpret_cast<const bf16x8*>(p);
  }
  static __device__ __forceinline__ void mma(const frag& a, const frag& b, f32x4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mfma<float> {
  struct frag {
    float4 lo, hi;
  };
  static __device__ __forceinline__ frag load(const float* p) {
    frag f;
    f.lo = *reinterpret_cast<const float4*>(p);
    f.hi = *reinterpret_cast<const float4*>(p + 4);
    return f;
  }
  // Eight k=4 products; in product j lane group g supplies k = 8g + j, so the
  // eight together cover the same 32 k values as one BF16 product.
  static __device__ __forceinline__ void mma(const frag& a, const frag& b, f32x4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo.x, b.lo.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo.y, b.lo.y, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo.z, b.lo.z, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.lo.w, b.lo.w, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi.x, b.hi.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi.y, b.hi.y, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi.z, b.hi.z, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.hi.w, b.hi.w, c, 0, 0, 0);
  }
};

template <class T>
__device__ __forceinline__ T to_t(float x) {
  return static_cast<T>(x);
}

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + __expf(-z)); }
// With the hardware reciprocal (about 1 ulp) instead of a correctly rounded
// divide: for activations that are rounded to BF16 next.
__device__ __forceinline__ float sigmoid_fast(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// Training noise (optional): noise[r][j] is added to input column c0 + j of
// batch row r before standardisation (and subtracted from the same target
// column by the loss).
struct Noise {
  const float* v;
  int64_t ld;
  int c0, n;
};

// EPI_LOSS: the output layer of a training pass with the loss in its epilogue.
enum Epi { EPI_HID = 0, EPI_OUT = 1, EPI_DX = 2, EPI_DW = 3, EPI_LOSS = 4 };

// The loss terms of EPI_LOSS (as the loss kernel takes them).
template <class T>
struct LossArgs {
  const float* y;
  int64_t ldy;
  const int* rows;
  int batch, n_out;
  const float* y_mean;
  const float* y_inv_std;
  float grad_scale;
  T* dY;
  int64_t lddy;
  T* dYT;
  int64_t lddyt;
  float* colsum;
  int ncols;
  double* partial;
  Noise nz;
};

template <class T>
struct GemmArgs {
  const T* A;
  const T* B;
  int64_t lda, ldb;
  int M, N, K;       // multiples of 64, 64, 32
  int k_split;       // K per grid.y slice (multiple of 32)
  const float* bias; // EPI_HID, EPI_OUT: [N]
  float* C;          // EPI_OUT: output; EPI_DW: partial dW slices
  T* Zt;             // EPI_HID: pre-activations Z, in the operand type (may be null)
  int64_t ldc;
  T* H;              // EPI_HID: activations; EPI_DX: dZ of the layer below
  int64_t ldh;
  T* HT;             // transposed copy of H (may be null)
  int64_t ldht;
  const T* Zin;      // EPI_DX: pre-activations of the layer below
  int64_t ldz;
  float* colsum;     // EPI_DX: per-64-row-tile column sums of dZ, [M/64][N]
  const float* scale;  // EPI_OUT: optional de-normalisation y*scale + shift
  const float* shift;
  int n_valid;       // EPI_OUT: columns written
  int m_valid;       // EPI_OUT: rows written
  LossArgs<T> loss;  // EPI_LOSS
};

// One block = 4 waves = one 64x64 output tile; wave w owns the 32x32 quadrant
// (w/2, w%2) as 2x2 MFMA blocks.  Blocks are renumbered so that the blocks one
// XCD receives (hardware deals them round-robin over 8 XCDs) are consecutive
// tiles, which share the A rows in that XCD's L2.
// LDS of one block: the two staged 64-wide chunks of A and B (BF16), reused
// after the products as the 64 x 64 FP32 output tile of the epilogue.
constexpr int GEMM_LDR = 64 + 8;                                  // staged row, elements
constexpr int GEMM_CT = TILE + 1;  // output tile row, floats (odd: rows and columns conflict-free)
constexpr int GEMM_SMEM = 2 * 2 * TILE * GEMM_LDR * 2;            // bytes
static_assert(TILE * GEMM_CT * 4 + 256 * 8 <= GEMM_SMEM,
              "output tile (and the loss epilogue's partial sums) fit the staging buffers");

// One 64 x 64 output tile `tile` of the product over K slice `slice`, with
// the block's LDS `smem` (GEMM_SMEM bytes).
template <class T, int EPI>
__device__ __forceinline__ void gemm_tile(const GemmArgs<T>& g, int tile, int slice,
                                          unsigned char* smem) {
  using M = Mfma<T>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tiles_n = g.N / TILE;
  const int mt = tile / tiles_n;
  const int m0 = mt * TILE + (wave >> 1) * 32;
  const int n0 = (tile % tiles_n) * TILE + (wave & 1) * 32;
  const int kb = slice * g.k_split;
  const int ke = min(g.K, kb + g.k_split);
  const int r16 = lane & 15, grp = lane >> 4;

  const T* a0 = g.A + (int64_t)(m0 + r16) * g.lda + grp * 8;
  const T* a1 = a0 + 16 * g.lda;
  const T* b0 = g.B + (int64_t)(n0 + r16) * g.ldb + grp * 8;
  const T* b1 = b0 + 16 * g.ldb;

  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  bool staged = false;
  if constexpr (std::is_same<T, __bf16>::value) {
    // BF16 with a K range of whole 64-wide chunks: the block stages each
    // chunk of its 64 A rows and 64 B rows in LDS (coalesced 16-byte loads,
    // eight lanes per row, two buffers, the next chunk's loads in flight
    // during the current chunk's products, one barrier per chunk), so a row
    // is fetched once per block rather than once per wave. In a chunk, lane
    // group grp takes k in [16 grp, 16 grp + 16) of its rows as two 8-element
    // slices and product j multiplies slice j of both operands; rows are
    // padded to 72 elements (eight lanes reading eight rows touch 32 banks).
    if (kb < ke && (ke - kb) % 64 == 0) {
      staged = true;
      constexpr int KC = 64, LDR = GEMM_LDR;
      auto As = reinterpret_cast<__bf16(*)[TILE][LDR]>(smem);
      auto Bs = As + 2;
      const int t = threadIdx.x;
      const int mb = mt * TILE, nbase = (tile % tiles_n) * TILE;
      bf16x8 ga[2], gb[2];
      auto fetch = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int piece = t + 256 * i, row = piece >> 3, c8 = (piece & 7) * 8;
          ga[i] = M::load(g.A + (int64_t)(mb + row) * g.lda + k0 + c8);
          gb[i] = M::load(g.B + (int64_t)(nbase + row) * g.ldb + k0 + c8);
        }
      };
      auto stage = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int piece = t + 256 * i, row = piece >> 3, c8 = (piece & 7) * 8;
          *reinterpret_cast<bf16x8*>(&As[buf][row][c8]) = ga[i];
          *reinterpret_cast<bf16x8*>(&Bs[buf][row][c8]) = gb[i];
        }
      };
      const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
      fetch(kb);
      stage(0);
      __syncthreads();
      const int n_chunks = (ke - kb) / KC;
      for (int c = 0; c < n_chunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < n_chunks) fetch(kb + (c + 1) * KC);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int kk = 16 * grp + 8 * j;
          const bf16x8 fa0 = *reinterpret_cast<const bf16x8*>(&As[buf][wm + r16][kk]);
          const bf16x8 fa1 = *reinterpret_cast<const bf16x8*>(&As[buf][wm + 16 + r16][kk]);
          const bf16x8 fb0 = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + r16][kk]);
          const bf16x8 fb1 = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + 16 + r16][kk]);
          M::mma(fa0, fb0, acc[0][0]);
          M::mma(fa0, fb1, acc[0][1]);
          M::mma(fa1, fb0, acc[1][0]);
          M::mma(fa1, fb1, acc[1][1]);
        }
        if (c + 1 < n_chunks) stage(buf ^ 1);
        __syncthreads();
      }
    }
  }

  if (kb < ke && !staged) {
    auto fa0 = M::load(a0 + kb), fa1 = M::load(a1 + kb);
    auto fb0 = M::load(b0 + kb), fb1 = M::load(b1 + kb);
    for (int k = kb + KSTEP; k < ke; k += KSTEP) {
      auto na0 = M::load(a0 + k), na1 = M::load(a1 + k);
      auto nb0 = M::load(b0 + k), nb1 = M::load(b1 + k);
      M::mma(fa0, fb0, acc[0][0]);
      M::mma(fa0, fb1, acc[0][1]);
      M::mma(fa1, fb0, acc[1][0]);
      M::mma(fa1, fb1, acc[1][1]);
      fa0 = na0; fa1 = na1; fb0 = nb0; fb1 = nb1;
    }
    M::mma(fa0, fb0, acc[0][0]);
    M::mma(fa0, fb1, acc[0][1]);
    M::mma(fa1, fb0, acc[1][0]);
    M::mma(fa1, fb1, acc[1][1]);
  }

  // ---- epilogue: acc[i][j][e] is C[m0 + 16i + 4 grp + e][n0 + 16j + r16]
  if constexpr (EPI == EPI_LOSS) {
    // The block holds every output column of its 64 rows (64 padded outputs):
    // yhat = acc + b goes through an LDS tile, then the same terms as the
    // loss kernel: L = mean over valid rows and the n_out columns of
    // (yhat - y_n)^2, y_n = (y - mean) / std; dL/dyhat row by row and its
    // transpose, the tile's column sums of it and the block's partial loss.
    const LossArgs<T>& q = g.loss;
    auto Ct = reinterpret_cast<float(*)[GEMM_CT]>(smem);
    double* lsum = reinterpret_cast<double*>(smem + TILE * GEMM_CT * 4);
    __syncthreads();  // the staged chunks are no longer read
    const int tr = (wave >> 1) * 32, tc = (wave & 1) * 32;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int e = 0; e < 4; ++e)
          Ct[tr + 16 * i + 4 * grp + e][tc + 16 * j + r16] =
              acc[i][j][e] + g.bias[n0 + 16 * j + r16];
    __syncthreads();
    const int t = threadIdx.x, c_t = t & 63, r_t = t >> 6;
    const int r0 = mt * TILE, c0 = (tile % tiles_n) * TILE;
    const int c = c0 + c_t;
    const bool cok = c < q.n_out;
    const bool noisy = q.nz.v && c >= q.nz.c0 && c < q.nz.c0 + q.nz.n;
    constexpr int RPT = 16;
    int64_t src[RPT];
    float yr[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = r0 + r_t + 4 * i;
      src[i] = r < q.batch ? (q.rows ? (int64_t)q.rows[r] : (int64_t)r) : -1;
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = r0 + r_t + 4 * i;
      yr[i] = (src[i] >= 0 && cok) ? q.y[src[i] * q.ldy + c] : 0.f;
      if (noisy && src[i] >= 0) yr[i] -= q.nz.v[(int64_t)r * q.nz.ld + (c - q.nz.c0)];
    }
    const float mu = cok ? q.y_mean[c] : 0.f, is = cok ? q.y_inv_std[c] : 0.f;
    double l2 = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int rr = r_t + 4 * i;
      float d = 0.f;
      if (src[i] >= 0 && cok) {
        const float e = Ct[rr][c_t] - (yr[i] - mu) * is;
        l2 += (double)e * e;
        d = q.grad_scale * e;
      }
      Ct[rr][c_t] = d;
      q.dY[(int64_t)(r0 + rr) * q.lddy + c] = to_t<T>(d);
    }
    lsum[t] = l2;
    __syncthreads();
    for (int cc = r_t; cc < 64; cc += 4)
      q.dYT[(int64_t)(c0 + cc) * q.lddyt + r0 + c_t] = to_t<T>(Ct[c_t][cc]);
    if (t < 64) {
      float sum = 0.f;
      for (int rr = 0; rr < 64; ++rr) sum += Ct[rr][t];
      q.colsum[(int64_t)mt * q.ncols + c0 + t] = sum;
    }
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) lsum[t] += lsum[t + w];
      __syncthreads();
    }
    if (t == 0) q.partial[(int64_t)(tile % tiles_n) * (g.M / TILE) + mt] = lsum[0];
  } else if constexpr (EPI == EPI_DW || EPI == EPI_OUT) {
    for (int i = 0; i < 2; ++i) {
      for (int j = 0; j < 2; ++j) {
        const int col = n0 + 16 * j + r16;
        const int row = m0 + 16 * i + 4 * grp;
        float v[4];
        for (int e = 0; e < 4; ++e) v[e] = acc[i][j][e];
        if constexpr (EPI == EPI_DW) {
          float* c = g.C + (int64_t)slice * g.M * g.ldc;
          for (int e = 0; e < 4; ++e) c[(int64_t)(row + e) * g.ldc + col] = v[e];
        } else {
          if (col < g.n_valid) {
            const float b = g.bias[col];
            float sc = 1.f, sh = 0.f;
            if (g.scale) {
              sc = g.scale[col];
              sh = g.shift[col];
            }
            for (int e = 0; e < 4; ++e)
              if (row + e < g.m_valid) g.C[(int64_t)(row + e) * g.ldc + col] = (v[e] + b) * sc + sh;
          }
        }
      }
    }
  } else {
    // Hidden-layer and input-gradient epilogues through LDS: the block's
    // 64 x 64 result goes to an FP32 tile, then every output (Z, the layer's
    // values H and their transpose HT) leaves as whole rows of 16-byte stores.
    // EPI_HID: z = acc + b, H = SiLU(z). EPI_DX: dz = acc silu'(z) with z read
    // from Zin row by row, then dz's column sums over the tile.
    auto Ct = reinterpret_cast<float(*)[GEMM_CT]>(smem);
    __syncthreads();  // the staged chunks are no longer read
    const int tr = (wave >> 1) * 32, tc = (wave & 1) * 32;  // this wave's quadrant
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int e = 0; e < 4; ++e) {
          float v = acc[i][j][e];
          if constexpr (EPI == EPI_HID) v += g.bias[n0 + 16 * j + r16];
          Ct[tr + 16 * i + 4 * grp + e][tc + 16 * j + r16] = v;
        }
    __syncthreads();
    const int t = threadIdx.x;
    const int mb = mt * TILE, nb = (tile % tiles_n) * TILE;
    constexpr int VEC = 16 / (int)sizeof(T);
    constexpr int PER = TILE * TILE / VEC / 256;  // 16-byte pieces per thread
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    if constexpr (EPI == EPI_HID) {
      if (g.Zt) {  // Z in the operand type, row by row
        for (int k = 0; k < PER; ++k) {
          const int piece = t + 256 * k;
          const int r = piece / (TILE / VEC), cv = (piece % (TILE / VEC)) * VEC;
          vec_t o;
          for (int q = 0; q < VEC; ++q) o[q] = to_t<T>(Ct[r][cv + q]);
          *reinterpret_cast<vec_t*>(g.Zt + (int64_t)(mb + r) * g.ldz + nb + cv) = o;
        }
      }
    } else {
      // dz in place: Zin read row by row, then its column sums
      for (int k = 0; k < PER; ++k) {
        const int piece = t + 256 * k;
        const int r = piece / (TILE / VEC), cv = (piece % (TILE / VEC)) * VEC;
        const vec_t z8 = *reinterpret_cast<const vec_t*>(g.Zin + (int64_t)(mb + r) * g.ldz + nb + cv);
        for (int q = 0; q < VEC; ++q) {
          const float z = (float)z8[q], sg = sigmoid(z);
          Ct[r][cv + q] *= sg * (1.f + z * (1.f - sg));
        }
      }
      __syncthreads();
      if (t < TILE) {
        float cs = 0.f;
        for (int r = 0; r < TILE; ++r) cs += Ct[r][t];
        g.colsum[(int64_t)mt * g.N + nb + t] = cs;
      }
    }
    // H row by row and HT column by column, VEC elements per 16-byte store
    auto out_val = [&](float v) __attribute__((always_inline)) {
      if constexpr (EPI == EPI_HID) return v * sigmoid(v);
      else return v;
    };
    for (int k = 0; k < PER; ++k) {
      const int piece = t + 256 * k;
      const int r = piece / (TILE / VEC), cv = (piece % (TILE / VEC)) * VEC;
      vec_t o;
      for (int q = 0; q < VEC; ++q) o[q] = to_t<T>(out_val(Ct[r][cv + q]));
      *reinterpret_cast<vec_t*>(g.H + (int64_t)(mb + r) * g.ldh + nb + cv) = o;
    }
    if (g.HT) {
      for (int k = 0; k < PER; ++k) {
        const int piece = t + 256 * k;
        const int c = piece / (TILE / VEC), rv = (piece % (TILE / VEC)) * VEC;
        vec_t o;
        for (int q = 0; q < VEC; ++q) o[q] = to_t<T>(out_val(Ct[rv + q][c]));
        *reinterpret_cast<vec_t*>(g.HT + (int64_t)(nb + c) * g.ldht + mb + rv) = o;
      }
    }
  }
}

// Blocks of one launch are renumbered so that the blocks one XCD receives
// (the hardware deals them round-robin over 8 XCDs) are consecutive tiles,
// which share the A rows in that XCD's L2 (when the count divides by 8).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

template <class T, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs<T> g) {
  __shared__ __align__(16) unsigned char smem[GEMM_SMEM];
  gemm_tile<T, EPI>(g, xcd_tile(blockIdx.x, gridDim.x), blockIdx.y, smem);
}

// The two products of one backward layer in one launch: they read the same
// dZ_l and are independent, so the input-gradient tiles (blocks [0, n_dx))
// and the weight-gradient tiles and slices (the rest, tile-major within a
// slice) run side by side instead of in two launches of a few hundred
// latency-bound blocks each.
template <class T>
__global__ __launch_bounds__(256) void gemm_pair_kernel(GemmArgs<T> dx, GemmArgs<T> dw, int n_dx,
                                                        int dw_tiles) {
  __shared__ __align__(16) unsigned char smem[GEMM_SMEM];
  const int b = blockIdx.x;
  if (b < n_dx) {
    gemm_tile<T, EPI_DX>(dx, xcd_tile(b, n_dx), 0, smem);
  } else {
    const int q = b - n_dx;
    gemm_tile<T, EPI_DW>(dw, q % dw_tiles, q / dw_tiles, smem);
  }
}

// Large-batch forward products (BF16 only): one block = 4 waves = a 128x128
// output tile, each wave 64x64 as 2x2 blocks of v_mfma_f32_32x32x16_bf16,
// which doubles the arithmetic per loaded byte of the 16x16 form. Lane l
// supplies row (l mod 32) and the k-slice 8*(l/32) .. +8 of both operands;
// the result lands as D[8*(e/4) + 4*(l/32) + (e mod 4)][l mod 32], e = 0..15.
// M and N must be multiples of 128, K of 32; EPI_HID or EPI_OUT.
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int BIG = 128;

template <int EPI>
__global__ __launch_bounds__(256) void gemm_big_kernel(GemmArgs<__bf16> g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tiles_n = g.N / BIG;
  int tile = blockIdx.x;
  const int nb = gridDim.x;
  if ((nb & 7) == 0) tile = (tile & 7) * (nb >> 3) + (tile >> 3);
  const int m0 = (tile / tiles_n) * BIG + (wave >> 1) * 64;
  const int n0 = (tile % tiles_n) * BIG + (wave & 1) * 64;
  const int r32 = lane & 31, grp = lane >> 5;
  // K is walked in chunks of 64. The block stages each chunk of its 128 A rows
  // and 128 B rows in LDS (coalesced 16-byte loads, eight lanes per row; the
  // next chunk's loads are in flight while the current one is multiplied,
  // two LDS buffers, one barrier per chunk), so a row is fetched once per
  // block rather than once per wave. In a chunk, lane (r32, grp) takes k in
  // [32 grp, 32 grp + 32) of its rows as four 8-element slices and product j
  // multiplies slice j of both operands: every k meets its partner once.
  // Rows are padded to 72 elements so that eight lanes reading eight rows
  // touch 32 distinct banks.
  constexpr int KC = 64, LDR = KC + 8;
  __shared__ __bf16 As[2][BIG][LDR];
  __shared__ __bf16 Bs[2][BIG][LDR];
  const int mt = (tile / tiles_n) * BIG, nt = (tile % tiles_n) * BIG;
  const int t = threadIdx.x;
  auto ld = [](const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); };
  bf16x8 ga[4], gb[4];
  auto fetch = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int piece = t + 256 * i, row = piece >> 3, c8 = (piece & 7) * 8;
      ga[i] = ld(g.A + (int64_t)(mt + row) * g.lda + k0 + c8);
      gb[i] = ld(g.B + (int64_t)(nt + row) * g.ldb + k0 + c8);
    }
  };
  auto stage = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int piece = t + 256 * i, row = piece >> 3, c8 = (piece & 7) * 8;
      *reinterpret_cast<bf16x8*>(&As[buf][row][c8]) = ga[i];
      *reinterpret_cast<bf16x8*>(&Bs[buf][row][c8]) = gb[i];
    }
  };
  f32x16 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  fetch(0);
  stage(0);
  __syncthreads();
  const int n_chunks = g.K / KC;
  for (int c = 0; c < n_chunks; ++c) {
    const int buf = c & 1;
    if (c + 1 < n_chunks) fetch((c + 1) * KC);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = 32 * grp + 8 * j;
      const bf16x8 fa0 = *reinterpret_cast<const bf16x8*>(&As[buf][wm + r32][kk]);
      const bf16x8 fa1 = *reinterpret_cast<const bf16x8*>(&As[buf][wm + 32 + r32][kk]);
      const bf16x8 fb0 = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + r32][kk]);
      const bf16x8 fb1 = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + 32 + r32][kk]);
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa0, fb0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa0, fb1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa1, fb0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa1, fb1, acc[1][1], 0, 0, 0);
    }
    if (c + 1 < n_chunks) stage(buf ^ 1);
    __syncthreads();
  }

  for (int i = 0; i < 2; ++i) {
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + 32 * j + r32;
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + 32 * i + 8 * q + 4 * grp;  // rows row .. row + 3
        if constexpr (EPI == EPI_OUT) {
          if (col < g.n_valid) {
            const float b = g.bias[col];
            float sc = 1.f, sh = 0.f;
            if (g.scale) {
              sc = g.scale[col];
              sh = g.shift[col];
            }
            for (int e = 0; e < 4; ++e)
              if (row + e < g.m_valid)
                g.C[(int64_t)(row + e) * g.ldc + col] = (acc[i][j][4 * q + e] + b) * sc + sh;
          }
        } else {
          const float b = g.bias[col];
          __bf16 out[4];
          for (int e = 0; e < 4; ++e) {
            const float z = acc[i][j][4 * q + e] + b;
            if (g.Zt) g.Zt[(int64_t)(row + e) * g.ldz + col] = (__bf16)z;
            out[e] = (__bf16)(z * sigmoid(z));
          }
          for (int e = 0; e < 4; ++e) g.H[(int64_t)(row + e) * g.ldh + col] = out[e];
          if (g.HT) {
            __bf16* ht = g.HT + (int64_t)col * g.ldht + row;
            for (int e = 0; e < 4; ++e) ht[e] = out[e];
          }
        }
      }
    }
  }
}

// ---- the whole forward pass of an inference network in one kernel ----------
// A block takes 128 input rows through every layer with the activations kept
// in LDS (BF16, rows padded by 8 elements against bank conflicts), so only
// the input rows and the outputs cross HBM. Eight waves, two per SIMD, so
// that one wave's matrix products overlap the other's activation epilogue.
// Hidden layer: wave w computes rows [64 (w / 4), + 64) x columns
// [(w % 4) NB 32, + NB 32) as 2 x NB blocks of v_mfma_f32_32x32x16_bf16, A
// from LDS, B (the weights, k-contiguous rows) straight from global memory
// in 64-wide K chunks with the next chunk's loads in flight (lane group g
// takes k in [32 g, 32 g + 32) of the chunk as four slices, product j the
// j-th slice of both operands); then every wave waits, writes SiLU(z) over
// the layer's input and waits again. Output layer (64 padded columns): wave w
// takes the 32 x 32 block (rows 32 (w / 2), columns 32 (w % 2)).
constexpr int MAX_LAYERS = 8;  // hidden layers + output layer
constexpr int FB_M = 128, FB_KMAX = 384, FB_LDA = FB_KMAX + 8, FB_WLD = 64 + 8;

struct FusedArgs {
  const __bf16* X;  // [M][ldx] standardised input rows (zero padded)
  int64_t ldx;
  int M, K0, H, n_hl;          // rows (multiple of 128), input width, hidden width (128 NB)
  const __bf16* W[MAX_LAYERS];  // layer l: [out_p][in_p] BF16, k contiguous
  int ldw[MAX_LAYERS];
  const float* b[MAX_LAYERS];
  float* y;  // [m_valid][ldy] de-standardised outputs
  int64_t ldy;
  int n_out, m_valid;
  const float* y_std;
  const float* y_mean;
};

template <int NB>
__global__ __launch_bounds__(512) void mlp_fused_kernel(FusedArgs f) {
  __shared__ __bf16 act[FB_M][FB_LDA];
  __shared__ __bf16 wst[FB_KMAX][FB_WLD];  // one 64-wide K chunk of a layer's weights
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = threadIdx.x;
  const int r32 = lane & 31, grp = lane >> 5;
  int blk = blockIdx.x;
  const int nb = gridDim.x;
  if ((nb & 7) == 0) blk = (blk & 7) * (nb >> 3) + (blk >> 3);
  const int m0 = blk * FB_M;
  auto ld8 = [](const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); };

  // input rows into LDS: 16-byte pieces, K0 / 8 per row
  {
    const int per_row = f.K0 / 8;
    for (int piece = t; piece < FB_M * per_row; piece += 512) {
      const int row = piece / per_row, c8 = (piece - row * per_row) * 8;
      *reinterpret_cast<bf16x8*>(&act[row][c8]) = ld8(f.X + (int64_t)(m0 + row) * f.ldx + c8);
    }
  }
  __syncthreads();

  const int r_base = (wave >> 2) * 64;
  constexpr int PIECES = 2 * NB;  // 16-byte pieces of a weight chunk per thread
  for (int l = 0; l < f.n_hl; ++l) {
    const int K = l == 0 ? f.K0 : f.H;
    const int n_base = (wave & 3) * NB * 32;
    // the layer's weights go through LDS in 64-wide K chunks (rows padded to
    // 72 elements), each 16-byte piece fetched once per block; the next
    // chunk's pieces are in registers while the current one is multiplied
    const __bf16* wl = f.W[l];
    const int ldw = f.ldw[l];
    bf16x8 stage[PIECES];
    auto fetch = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
      for (int i = 0; i < PIECES; ++i) {
        const int piece = t + 512 * i, row = piece >> 3, c8 = (piece & 7) * 8;
        stage[i] = ld8(wl + (int64_t)row * ldw + k0 + c8);
      }
    };
    f32x16 acc[2][NB];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int c = 0; c < NB; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[i][c][e] = 0.f;
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += 64) {
      __syncthreads();  // the previous chunk's weights are no longer read
#pragma unroll
      for (int i = 0; i < PIECES; ++i) {
        const int piece = t + 512 * i, row = piece >> 3, c8 = (piece & 7) * 8;
        *reinterpret_cast<bf16x8*>(&wst[row][c8]) = stage[i];
      }
      __syncthreads();
      if (k0 + 64 < K) fetch(k0 + 64);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int kk = 32 * grp + 8 * j;
        bf16x8 fb[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c)
          fb[c] = *reinterpret_cast<const bf16x8*>(&wst[n_base + 32 * c + r32][kk]);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&act[r_base + 32 * i + r32][k0 + kk]);
#pragma unroll
          for (int c = 0; c < NB; ++c)
            acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb[c], acc[i][c], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // every wave has read the layer's input
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const int col = n_base + 32 * c + r32;
      const float bc = f.b[l][col];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float z = acc[i][c][4 * q + e] + bc;
            act[r_base + 32 * i + 8 * q + 4 * grp + e][col] = (__bf16)(z * sigmoid_fast(z));
          }
    }
    __syncthreads();  // the layer's output is complete
  }

  // output layer: 64 padded columns, 32 x 32 per wave
  {
    const int L = f.n_hl;
    const int ro = 32 * (wave >> 1), co = 32 * (wave & 1);
    const __bf16* w0 = f.W[L] + (int64_t)(co + r32) * f.ldw[L] + grp * 32;
    f32x16 acc;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0.f;
    for (int k0 = 0; k0 < f.H; k0 += 64) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int kk = k0 + 32 * grp + 8 * j;
        const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&act[ro + r32][kk]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, ld8(w0 + k0 + 8 * j), acc, 0, 0, 0);
      }
    }
    const int col = co + r32;
    if (col < f.n_out) {
      const float bc = f.b[L][col], sc = f.y_std[col], sh = f.y_mean[col];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = m0 + ro + 8 * q + 4 * grp + e;
          if (row < f.m_valid) f.y[(int64_t)row * f.ldy + col] = (acc[4 * q + e] + bc) * sc + sh;
        }
    }
  }
}

// ---- layer-0 input: gather rows, standardise, pad, write X and X^T ---------
// Block: 64 rows x 64 columns through an LDS tile.
template <class T>
__global__ __launch_bounds__(256) void pack_input_kernel(
    const float* __restrict__ x, int64_t ldx, const int* __restrict__ rows, int batch, int n_in,
    const float* __restrict__ mean, const float* __restrict__ inv_std, T* X, int64_t ldX, T* XT,
    int64_t ldXT, Noise nz) {
  __shared__ float tile[64][65];
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  const int tc = threadIdx.x & 63, tr = threadIdx.x >> 6;
  const int c = c0 + tc;
  const bool cok = c < n_in;
  const bool noisy = nz.v && c >= nz.c0 && c < nz.c0 + nz.n;
  // a thread's 16 rows: every gather index, then every load, are issued
  // before the first use, so the dependent loads overlap
  constexpr int RPT = 16;
  int64_t src[RPT];
  float xr[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = r0 + tr + 4 * i;
    src[i] = r < batch ? (rows ? (int64_t)rows[r] : (int64_t)r) : -1;
  }
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = r0 + tr + 4 * i;
    xr[i] = (src[i] >= 0 && cok) ? x[src[i] * ldx + c] : 0.f;
    if (noisy && src[i] >= 0) xr[i] += nz.v[(int64_t)r * nz.ld + (c - nz.c0)];
  }
  const float mu = cok ? mean[c] : 0.f, is = cok ? inv_std[c] : 0.f;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int rr = tr + 4 * i;
    const float v = (src[i] >= 0 && cok) ? (xr[i] - mu) * is : 0.f;
    tile[rr][tc] = v;
    X[(int64_t)(r0 + rr) * ldX + c] = to_t<T>(v);
  }
  if (!XT) return;
  __syncthreads();
  for (int cc = tr; cc < 64; cc += 4) XT[(int64_t)(c0 + cc) * ldXT + r0 + tc] = to_t<T>(tile[tc][cc]);
}

// ---- the loss's partial sums (the output layer's epilogue writes one per block)
__global__ void loss_final_kernel(const double* partial, int n, double inv_count, float* out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += partial[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(s[0] * inv_count);
}

// ---- parameter-vector kernels ----------------------------------------------
// The padded parameter vector holds, per layer, W [out_p][in_p] then b [out_p].
struct LayerTable {
  int n_layers;
  int64_t off[MAX_LAYERS + 1];  // start of each layer's block in the padded vector
  int in_p[MAX_LAYERS], out_p[MAX_LAYERS];
  int in_r[MAX_LAYERS], out_r[MAX_LAYERS];       // real sizes
  int64_t off_r[MAX_LAYERS + 1];                 // same in the unpadded vector
  int64_t woff[MAX_LAYERS];      // start of each layer's operand copy W (and W^T)
  const float* dwp[MAX_LAYERS];  // split-K weight-gradient slices [slices][out_p][in_p]
  int dw_slices[MAX_LAYERS];
  const float* dbp[MAX_LAYERS];  // bias-gradient tile sums [tiles][out_p]
  int db_tiles;
};

__device__ __forceinline__ int layer_of(const LayerTable& t, int64_t p) {
  int l = 0;
  while (l + 1 < t.n_layers && p >= t.off[l + 1]) ++l;
  return l;
}

// g[p] = sum of the partial gradients of parameter p (fixed order).
__global__ void grad_reduce_kernel(LayerTable t, float* g) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= t.off[t.n_layers]) return;
  const int l = layer_of(t, p);
  const int64_t q = p - t.off[l];
  const int64_t nw = (int64_t)t.out_p[l] * t.in_p[l];
  float s = 0.f;
  // (unrolled so that the loads of a run of slices are in flight together;
  // the additions keep their order)
  if (q < nw) {
#pragma unroll 8
    for (int k = 0; k < t.dw_slices[l]; ++k) s += t.dwp[l][(int64_t)k * nw + q];
  } else {
    const int o = (int)(q - nw);
#pragma unroll 8
    for (int k = 0; k < t.db_tiles; ++k) s += t.dbp[l][(int64_t)k * t.out_p[l] + o];
  }
  g[p] = s;
}

// Adam on the FP32 master vector (update != 0), then the operand copies of
// the weights, W [out_p][in_p] and W^T [in_p][out_p], from the master values.
template <class T>
__global__ void adam_kernel(LayerTable t, int update, float* P, const float* G, float* Mom,
                            float* Vel, float lr, float b1, float b2, float eps, float c1, float c2,
                            T* Wc, T* WTc) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= t.off[t.n_layers]) return;
  float w = P[p];
  if (update) {
    const float gr = G[p];
    const float m = b1 * Mom[p] + (1.f - b1) * gr;
    const float v = b2 * Vel[p] + (1.f - b2) * gr * gr;
    Mom[p] = m;
    Vel[p] = v;
    w -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    P[p] = w;
  }
  const int l = layer_of(t, p);
  const int64_t q = p - t.off[l];
  const int64_t nw = (int64_t)t.out_p[l] * t.in_p[l];
  if (q < nw) {
    const int o = (int)(q / t.in_p[l]), i = (int)(q % t.in_p[l]);
    Wc[t.woff[l] + q] = to_t<T>(w);
    WTc[t.woff[l] + (int64_t)i * t.out_p[l] + o] = to_t<T>(w);
  }
}

// One training step's parameter update in one pass: the gradient of p as
// grad_reduce_kernel sums it (same order, so the same bits), kept in G, then
// Adam as adam_kernel takes it (c1 = 1 - b1^t, c2 = 1 - b2^t), then the
// operand copies.
// Block 0 also sums the loss kernel's partial losses (`n_part` of them, the
// same order as loss_final_kernel) into loss_out[0] when loss_out is set.
template <class T>
__global__ __launch_bounds__(256) void reduce_adam_kernel(
    LayerTable t, float* G, float* P, float* Mom, float* Vel, float lr, float b1, float b2,
    float eps, float c1, float c2, T* Wc, T* WTc, const double* loss_part, int n_part,
    double inv_count, float* loss_out) {
  if (blockIdx.x == 0 && loss_out) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n_part; i += 256) acc += loss_part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) loss_out[0] = (float)(s[0] * inv_count);
  }
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= t.off[t.n_layers]) return;
  const int l = layer_of(t, p);
  const int64_t q = p - t.off[l];
  const int64_t nw = (int64_t)t.out_p[l] * t.in_p[l];
  float gr = 0.f;
  if (q < nw) {
#pragma unroll 8
    for (int k = 0; k < t.dw_slices[l]; ++k) gr += t.dwp[l][(int64_t)k * nw + q];
  } else {
    const int o = (int)(q - nw);
#pragma unroll 8
    for (int k = 0; k < t.db_tiles; ++k) gr += t.dbp[l][(int64_t)k * t.out_p[l] + o];
  }
  G[p] = gr;
  const float m = b1 * Mom[p] + (1.f - b1) * gr;
  const float v = b2 * Vel[p] + (1.f - b2) * gr * gr;
  Mom[p] = m;
  Vel[p] = v;
  const float w = P[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  P[p] = w;
  if (q < nw) {
    const int o = (int)(q / t.in_p[l]), i = (int)(q % t.in_p[l]);
    Wc[t.woff[l] + q] = to_t<T>(w);
    WTc[t.woff[l] + (int64_t)i * t.out_p[l] + o] = to_t<T>(w);
  }
}

// Between the padded vector and the unpadded flat order (per layer W [out][in]
// row-major, then b [out]).  dir 0: padded -> flat, 1: flat -> padded.
__global__ void repack_kernel(LayerTable t, int dir, float* padded, float* flat) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= t.off[t.n_layers]) return;
  const int l = layer_of(t, p);
  const int64_t q = p - t.off[l];
  const int64_t nw = (int64_t)t.out_p[l] * t.in_p[l];
  int64_t f = -1;
  if (q < nw) {
    const int o = (int)(q / t.in_p[l]), i = (int)(q % t.in_p[l]);
    if (o < t.out_r[l] && i < t.in_r[l]) f = t.off_r[l] + (int64_t)o * t.in_r[l] + i;
  } else {
    const int o = (int)(q - nw);
    if (o < t.out_r[l]) f = t.off_r[l] + (int64_t)t.out_r[l] * t.in_r[l] + o;
  }
  if (dir == 0) {
    if (f >= 0) flat[f] = padded[p];
  } else {
    padded[p] = f >= 0 ? flat[f] : 0.f;
  }
}

// ---- column statistics (FP64 accumulation) ---------------------------------
// partial[b][c] = sum over rows [b*chunk, (b+1)*chunk) of (x - shift[c])^pow
__global__ void colstat_kernel(const float* __restrict__ x, int64_t ldx, int64_t rows, int cols,
                               int64_t chunk, const double* shift, int pw, double* partial) {
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min(rows, r0 + chunk);
  for (int c = threadIdx.x; c < cols; c += blockDim.x) {
    const double sh = shift ? shift[c] : 0.0;
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const double d = (double)x[r * ldx + c] - sh;
      s += pw == 1 ? d : d * d;
    }
    partial[(int64_t)blockIdx.x * cols + c] = s;
  }
}

__global__ void colstat_final_kernel(const double* partial, int nb, int cols, double inv_rows,
                                     int take_sqrt, double* out, float* out_f) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * cols + c];
  s *= inv_rows;
  if (take_sqrt) s = sqrt(s);
  out[c] = s;
  out_f[c] = (float)s;
}

}  // namespace

// ============================================================================
// Host side
// ============================================================================

struct npx_sur {
  int device = 0;
  int n_in = 0, n_hidden = 0, n_hl = 0, n_out = 0, max_batch = 0, precision = 0, training = 0;
  int n_layers = 0, hp = 0, in_p0 = 0, out_p = 0, Mp_max = 0;
  size_t esz = 2;  // operand element size
  LayerTable tab{};
  int64_t n_pad = 0, n_real = 0, n_wc = 0;
  int step = 0;
  double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  Noise noise{nullptr, 0, 0, 0};

  // parameters: master, gradient, Adam moments (padded order), operand copies
  float *P = nullptr, *G = nullptr, *Mom = nullptr, *Vel = nullptr, *flat = nullptr;
  void *Wc = nullptr, *WTc = nullptr;
  // standardisation
  float *x_mean = nullptr, *x_inv = nullptr, *y_mean = nullptr, *y_inv = nullptr, *y_std = nullptr;
  // activations
  void* X0 = nullptr;
  void* X0T = nullptr;
  std::vector<void*> H, HT;
  std::vector<void*> Z;  // pre-activations, in the operand type
  void *dA = nullptr, *dAT = nullptr, *dB = nullptr, *dBT = nullptr;
  std::vector<float*> dwp, dbp;
  double* loss_part = nullptr;
  float* loss_tmp = nullptr;
  std::vector<void*> owned;
};

namespace {

constexpr int MAX_SLICES = 32;

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

template <class P>
hipError_t sur_alloc(npx_sur* s, P** p, size_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
  if (e == hipSuccess) {
    s->owned.push_back(q);
    *p = static_cast<P*>(q);
  }
  return e;
}

void sur_free(npx_sur* s) {
  for (void* q : s->owned) (void)hipFree(q);
  s->owned.clear();
}

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int k_slices(int tiles, int K) {
  int s = std::max(1, std::min(MAX_SLICES, (512 + tiles - 1) / tiles));
  s = std::min(s, std::max(1, K / 256));
  return s;
}

template <class T, int EPI>
hipError_t launch_gemm(const GemmArgs<T>& g, int slices, hipStream_t st) {
  if (g.M % TILE || g.N % TILE || g.K % KSTEP || g.k_split % KSTEP ||
      (int64_t)g.k_split * slices < g.K)
    return hipErrorInvalidValue;
  // large forward products: 128x128 tiles when they give at least 4 blocks per CU
  if constexpr (std::is_same<T, __bf16>::value && (EPI == EPI_HID || EPI == EPI_OUT)) {
    if (slices == 1 && g.M % BIG == 0 && g.N % BIG == 0 && g.K % 64 == 0 &&
        (g.M / BIG) * (g.N / BIG) >= 1024) {
      hipLaunchKernelGGL((gemm_big_kernel<EPI>), dim3((g.M / BIG) * (g.N / BIG)), dim3(256), 0,
                         st, g);
      return hipGetLastError();
    }
  }
  dim3 grid((g.M / TILE) * (g.N / TILE), slices);
  hipLaunchKernelGGL((gemm_kernel<T, EPI>), grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

// The input-gradient product `dx` (one slice) and the weight-gradient product
// `dw` (in `slices` K slices) of one backward layer, as one launch.
template <class T>
hipError_t launch_gemm_pair(const GemmArgs<T>& dx, const GemmArgs<T>& dw, int slices,
                            hipStream_t st) {
  auto ok = [](const GemmArgs<T>& g, int sl) {
    return !(g.M % TILE || g.N % TILE || g.K % KSTEP || g.k_split % KSTEP ||
             (int64_t)g.k_split * sl < g.K);
  };
  if (!ok(dx, 1) || !ok(dw, slices) || dx.k_split < dx.K) return hipErrorInvalidValue;
  const int n_dx = (dx.M / TILE) * (dx.N / TILE), dw_tiles = (dw.M / TILE) * (dw.N / TILE);
  hipLaunchKernelGGL((gemm_pair_kernel<T>), dim3(n_dx + dw_tiles * slices), dim3(256), 0, st, dx,
                     dw, n_dx, dw_tiles);
  return hipGetLastError();
}

template <class T>
GemmArgs<T> gemm_args(const void* A, int64_t lda, const void* B, int64_t ldb, int M, int N, int K) {
  GemmArgs<T> g{};
  g.A = static_cast<const T*>(A);
  g.B = static_cast<const T*>(B);
  g.lda = lda;
  g.ldb = ldb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.k_split = K;
  return g;
}

template <class T>
const T* wc(const npx_sur* s, int l) {
  return static_cast<const T*>(s->Wc) + s->tab.woff[l];
}
template <class T>
const T* wtc(const npx_sur* s, int l) {
  return static_cast<const T*>(s->WTc) + s->tab.woff[l];
}
inline const float* bias(const npx_sur* s, int l) {
  return s->P + s->tab.off[l] + (int64_t)s->tab.out_p[l] * s->tab.in_p[l];
}

// Forward pass over `batch` gathered rows.  final_out == nullptr: training
// pass through the hidden layers (pre-activations and transposed copies; the
// training pass runs the output layer with the loss in its epilogue); else
// the de-normalised prediction goes to final_out.
template <class T>
npx_status forward_packed_t(npx_sur* s, int batch, float* final_out, int64_t ld_out,
                            hipStream_t st);

template <class T>
npx_status forward_t(npx_sur* s, const float* x, int64_t ldx, const int* rows, int batch,
                     float* final_out, int64_t ld_out, hipStream_t st) {
  const int Mp = round_up(batch, TILE);
  const bool train = final_out == nullptr;
  dim3 grid(Mp / TILE, s->in_p0 / TILE);
  hipLaunchKernelGGL((pack_input_kernel<T>), grid, dim3(256), 0, st, x, ldx, rows, batch,
                     s->n_in, s->x_mean, s->x_inv, static_cast<T*>(s->X0), (int64_t)s->in_p0,
                     train ? static_cast<T*>(s->X0T) : nullptr, (int64_t)Mp,
                     train ? s->noise : Noise{nullptr, 0, 0, 0});
  HIP_TRY(hipGetLastError());
  return forward_packed_t<T>(s, batch, final_out, ld_out, st);
}

// The layers from the packed, standardised input rows in X0 (and X0T when
// training) onwards.
template <class T>
npx_status forward_packed_t(npx_sur* s, int batch, float* final_out, int64_t ld_out,
                            hipStream_t st) {
  const int Mp = round_up(batch, TILE);
  const bool train = final_out == nullptr;
  if constexpr (std::is_same<T, __bf16>::value) {
    // inference over whole 128-row blocks of a network whose widths fit the
    // fused kernel: one launch for all layers
    const int nb = s->hp / 128;
    if (!train && Mp % FB_M == 0 && s->hp % 128 == 0 && nb >= 1 && nb <= 3 &&
        s->in_p0 <= FB_KMAX && s->out_p == 64 && s->n_hl >= 1 && s->n_layers <= MAX_LAYERS) {
      FusedArgs f{};
      f.X = static_cast<const __bf16*>(s->X0);
      f.ldx = s->in_p0;
      f.M = Mp;
      f.K0 = s->in_p0;
      f.H = s->hp;
      f.n_hl = s->n_hl;
      for (int l = 0; l < s->n_layers; ++l) {
        f.W[l] = wc<__bf16>(s, l);
        f.ldw[l] = s->tab.in_p[l];
        f.b[l] = bias(s, l);
      }
      f.y = final_out;
      f.ldy = ld_out;
      f.n_out = s->n_out;
      f.m_valid = batch;
      f.y_std = s->y_std;
      f.y_mean = s->y_mean;
      const dim3 grid(Mp / FB_M), block(512);
      switch (nb) {
        case 1: hipLaunchKernelGGL(mlp_fused_kernel<1>, grid, block, 0, st, f); break;
        case 2: hipLaunchKernelGGL(mlp_fused_kernel<2>, grid, block, 0, st, f); break;
        default: hipLaunchKernelGGL(mlp_fused_kernel<3>, grid, block, 0, st, f); break;
      }
      HIP_TRY(hipGetLastError());
      return NPX_OK;
    }
  }
  const void* prev = s->X0;
  int64_t ld_prev = s->in_p0;
  for (int l = 0; l < s->n_hl; ++l) {
    GemmArgs<T> g = gemm_args<T>(prev, ld_prev, wc<T>(s, l), s->tab.in_p[l], Mp, s->hp,
                                 s->tab.in_p[l]);
    g.bias = bias(s, l);
    g.Zt = train ? static_cast<T*>(s->Z[l]) : nullptr;
    g.ldz = s->hp;
    g.H = static_cast<T*>(s->H[l]);
    g.ldh = s->hp;
    g.HT = train ? static_cast<T*>(s->HT[l]) : nullptr;
    g.ldht = Mp;
    HIP_TRY((launch_gemm<T, EPI_HID>(g, 1, st)));
    prev = s->H[l];
    ld_prev = s->hp;
  }
  if (train) return NPX_OK;  // the training pass runs the output layer with its loss
  const int L = s->n_layers - 1;
  GemmArgs<T> g = gemm_args<T>(prev, ld_prev, wc<T>(s, L), s->tab.in_p[L], Mp, s->out_p,
                               s->tab.in_p[L]);
  g.bias = bias(s, L);
  g.C = final_out;
  g.ldc = ld_out;
  g.n_valid = s->n_out;
  g.m_valid = batch;
  g.scale = s->y_std;
  g.shift = s->y_mean;
  HIP_TRY((launch_gemm<T, EPI_OUT>(g, 1, st)));
  return NPX_OK;
}

// Loss and gradient into G (padded order); loss (mean squared error over the
// batch and the n_out standardised outputs) to loss_out[0].
template <class T>
npx_status backward_t(npx_sur* s, const float* x, int64_t ldx, const float* y, int64_t ldy,
                      const int* rows, int batch, float* loss_out, hipStream_t st,
                      bool reduce = true) {
  npx_status r = forward_t<T>(s, x, ldx, rows, batch, nullptr, 0, st);
  if (r != NPX_OK) return r;
  const int Mp = round_up(batch, TILE);
  const int tiles_m = Mp / TILE;
  const int L = s->n_layers - 1;
  {
    // the output layer with the loss in its epilogue: dL/dyhat (and its
    // transpose), the output bias gradient's tile sums, the partial losses
    const void* hin = s->n_hl > 0 ? s->H[s->n_hl - 1] : s->X0;
    const int64_t ld_in = s->n_hl > 0 ? s->hp : s->in_p0;
    GemmArgs<T> g = gemm_args<T>(hin, ld_in, wc<T>(s, L), s->tab.in_p[L], Mp, s->out_p,
                                 s->tab.in_p[L]);
    g.bias = bias(s, L);
    LossArgs<T>& q = g.loss;
    q.y = y;
    q.ldy = ldy;
    q.rows = rows;
    q.batch = batch;
    q.n_out = s->n_out;
    q.y_mean = s->y_mean;
    q.y_inv_std = s->y_inv;
    q.grad_scale = 2.0f / ((float)batch * (float)s->n_out);
    q.dY = static_cast<T*>(s->dA);
    q.lddy = s->out_p;
    q.dYT = static_cast<T*>(s->dAT);
    q.lddyt = Mp;
    q.colsum = s->dbp[L];
    q.ncols = s->out_p;
    q.partial = s->loss_part;
    q.nz = s->noise;
    HIP_TRY((launch_gemm<T, EPI_LOSS>(g, 1, st)));
    // the training step sums the partial losses inside its update
    if (reduce) {
      hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, s->loss_part,
                         tiles_m * (s->out_p / TILE), 1.0 / ((double)batch * s->n_out),
                         loss_out ? loss_out : s->loss_tmp);
      HIP_TRY(hipGetLastError());
    }
  }
  void *cur = s->dA, *curT = s->dAT, *nxt = s->dB, *nxtT = s->dBT;
  for (int l = L; l >= 0; --l) {
    const int out_p = s->tab.out_p[l], in_p = s->tab.in_p[l];
    // dW_l = dZ_l^T * H_{l-1}, split over the batch
    const void* hprevT = l == 0 ? s->X0T : s->HT[l - 1];
    GemmArgs<T> gw = gemm_args<T>(curT, Mp, hprevT, Mp, out_p, in_p, Mp);
    const int tiles = (out_p / TILE) * (in_p / TILE);
    const int sl = k_slices(tiles, Mp);
    gw.k_split = round_up((Mp + sl - 1) / sl, 64);  // whole 64-wide chunks (LDS-staged)
    const int used = (Mp + gw.k_split - 1) / gw.k_split;
    gw.C = s->dwp[l];
    gw.ldc = in_p;
    s->tab.dw_slices[l] = used;
    if (l == 0) {
      HIP_TRY((launch_gemm<T, EPI_DW>(gw, used, st)));
      break;
    }
    // dZ_{l-1} = (dZ_l * W_l) . silu'(Z_{l-1}), in the same launch as dW_l
    GemmArgs<T> gx = gemm_args<T>(cur, out_p, wtc<T>(s, l), out_p, Mp, in_p, out_p);
    gx.Zin = static_cast<const T*>(s->Z[l - 1]);
    gx.ldz = s->hp;
    gx.H = static_cast<T*>(nxt);
    gx.ldh = in_p;
    gx.HT = static_cast<T*>(nxtT);
    gx.ldht = Mp;
    gx.colsum = s->dbp[l - 1];
    HIP_TRY((launch_gemm_pair<T>(gx, gw, used, st)));
    std::swap(cur, nxt);
    std::swap(curT, nxtT);
  }
  s->tab.db_tiles = tiles_m;
  for (int l = 0; l <= L; ++l) {
    s->tab.dwp[l] = s->dwp[l];
    s->tab.dbp[l] = s->dbp[l];
  }
  if (!reduce) return NPX_OK;  // the training step reduces inside its update
  const int blocks = (int)((s->n_pad + 255) / 256);
  hipLaunchKernelGGL(grad_reduce_kernel, dim3(blocks), dim3(256), 0, st, s->tab, s->G);
  HIP_TRY(hipGetLastError());
  return NPX_OK;
}

template <class T>
hipError_t refresh_t(npx_sur* s, int update, float lr, hipStream_t st) {
  const int blocks = (int)((s->n_pad + 255) / 256);
  float c1 = 1.f, c2 = 1.f;
  if (update) {
    c1 = (float)(1.0 - std::pow(s->b1, s->step));
    c2 = (float)(1.0 - std::pow(s->b2, s->step));
  }
  hipLaunchKernelGGL((adam_kernel<T>), dim3(blocks), dim3(256), 0, st, s->tab, update, s->P,
                     s->G, s->Mom, s->Vel, lr, (float)s->b1, (float)s->b2, (float)s->eps, c1, c2,
                     static_cast<T*>(s->Wc), static_cast<T*>(s->WTc));
  return hipGetLastError();
}

hipError_t refresh(npx_sur* s, int update, float lr, hipStream_t st) {
  return s->precision == NPX_SUR_FP32 ? refresh_t<float>(s, update, lr, st)
                                      : refresh_t<__bf16>(s, update, lr, st);
}

npx_status check_io(const npx_sur* s, const float* x, int64_t ldx, int64_t batch) {
  if (!s) return fail(NPX_EINVAL, "null surrogate handle");
  if (batch < 0 || batch > s->max_batch)
    return fail(NPX_EINVAL, "batch %lld outside [0, %d]", (long long)batch, s->max_batch);
  if (batch > 0 && !x) return fail(NPX_EINVAL, "null input");
  if (ldx < s->n_in) return fail(NPX_EINVAL, "input row stride %lld < n_in %d", (long long)ldx, s->n_in);
  return NPX_OK;
}

}  // namespace

namespace npx {
npx_status sur_input(npx_sur* s, int batch, SurInput* in) {
  if (!s) return fail(NPX_EINVAL, "null surrogate handle");
  if (batch < 0 || batch > s->max_batch)
    return fail(NPX_EINVAL, "batch %d outside [0, %d]", batch, s->max_batch);
  in->x = s->X0;
  in->ld = s->in_p0;
  in->width = s->in_p0;
  in->rows = round_up(batch, TILE);
  in->mean = s->x_mean;
  in->inv_std = s->x_inv;
  in->bf16 = s->precision != NPX_SUR_FP32;
  return NPX_OK;
}

npx_status sur_forward_input(npx_sur* s, int batch, float* y, int64_t ldy, hipStream_t st) {
  if (!s) return fail(NPX_EINVAL, "null surrogate handle");
  if (batch == 0) return NPX_OK;
  if (!y || ldy < s->n_out) return fail(NPX_EINVAL, "bad output buffer or stride");
  return s->precision == NPX_SUR_FP32 ? forward_packed_t<float>(s, batch, y, ldy, st)
                                      : forward_packed_t<__bf16>(s, batch, y, ldy, st);
}

void sur_dims(const npx_sur* s, int* n_in, int* n_out, int* max_batch) {
  *n_in = s->n_in;
  *n_out = s->n_out;
  *max_batch = s->max_batch;
}
}  // namespace npx

extern "C" {

npx_status npx_sur_create(const npx_sur_desc* d, npx_sur** out) {
  if (!d || !out) return fail(NPX_EINVAL, "null argument");
  *out = nullptr;
  if (d->n_in < 1 || d->n_hidden < 1 || d->n_out < 1 || d->n_hidden_layers < 1 ||
      d->n_hidden_layers >= MAX_LAYERS || d->max_batch < 1 || d->max_batch > (1 << 24))
    return fail(NPX_EINVAL, "bad network shape or batch limit");
  if (d->precision != NPX_SUR_BF16 && d->precision != NPX_SUR_FP32)
    return fail(NPX_EINVAL, "precision must be NPX_SUR_BF16 or NPX_SUR_FP32");
  npx_sur* s = new npx_sur();
  (void)hipGetDevice(&s->device);
  s->n_in = d->n_in;
  s->n_hidden = d->n_hidden;
  s->n_hl = d->n_hidden_layers;
  s->n_out = d->n_out;
  s->max_batch = d->max_batch;
  s->precision = d->precision;
  s->training = d->training != 0;
  s->esz = s->precision == NPX_SUR_FP32 ? 4 : 2;
  s->n_layers = s->n_hl + 1;
  s->hp = round_up(s->n_hidden, TILE);
  s->in_p0 = round_up(s->n_in, TILE);
  s->out_p = round_up(s->n_out, TILE);
  s->Mp_max = round_up(s->max_batch, TILE);
  LayerTable& t = s->tab;
  t.n_layers = s->n_layers;
  int64_t off = 0, off_r = 0, woff = 0;
  for (int l = 0; l < s->n_layers; ++l) {
    t.in_p[l] = l == 0 ? s->in_p0 : s->hp;
    t.out_p[l] = l == s->n_layers - 1 ? s->out_p : s->hp;
    t.in_r[l] = l == 0 ? s->n_in : s->n_hidden;
    t.out_r[l] = l == s->n_layers - 1 ? s->n_out : s->n_hidden;
    t.off[l] = off;
    t.off_r[l] = off_r;
    t.woff[l] = woff;
    off += (int64_t)t.out_p[l] * (t.in_p[l] + 1);
    off_r += (int64_t)t.out_r[l] * (t.in_r[l] + 1);
    woff += (int64_t)t.out_p[l] * t.in_p[l];
  }
  t.off[s->n_layers] = off;
  t.off_r[s->n_layers] = off_r;
  s->n_pad = off;
  s->n_real = off_r;
  s->n_wc = woff;

  // initial weights and biases: U(-1/sqrt(fan_in), 1/sqrt(fan_in)), padding 0
  std::vector<float> hostP((size_t)s->n_pad, 0.f);
  uint64_t rs = d->seed;
  for (int l = 0; l < s->n_layers; ++l) {
    const double bound = 1.0 / std::sqrt((double)t.in_r[l]);
    float* w = hostP.data() + t.off[l];
    for (int o = 0; o < t.out_r[l]; ++o)
      for (int i = 0; i < t.in_r[l]; ++i)
        w[(int64_t)o * t.in_p[l] + i] =
            (float)(bound * (2.0 * ((splitmix64(rs) >> 11) * 0x1.0p-53) - 1.0));
    float* b = w + (int64_t)t.out_p[l] * t.in_p[l];
    for (int o = 0; o < t.out_r[l]; ++o)
      b[o] = (float)(bound * (2.0 * ((splitmix64(rs) >> 11) * 0x1.0p-53) - 1.0));
  }

  const size_t Mp = (size_t)s->Mp_max;
  hipError_t e = hipSuccess;
  auto A = [&](auto** p, size_t bytes) {
    if (e == hipSuccess) e = sur_alloc(s, p, bytes);
  };
  A(&s->P, s->n_pad * 4);
  A(&s->G, s->n_pad * 4);
  A(&s->Mom, s->n_pad * 4);
  A(&s->Vel, s->n_pad * 4);
  A(&s->flat, s->n_real * 4);
  A(&s->Wc, s->n_wc * s->esz);
  A(&s->WTc, s->n_wc * s->esz);
  A(&s->x_mean, s->n_in * 4);
  A(&s->x_inv, s->n_in * 4);
  A(&s->y_mean, s->n_out * 4);
  A(&s->y_inv, s->n_out * 4);
  A(&s->y_std, s->n_out * 4);
  A(&s->X0, Mp * s->in_p0 * s->esz);
  s->H.assign(s->n_hl, nullptr);
  for (int l = 0; l < s->n_hl; ++l) A(&s->H[l], Mp * s->hp * s->esz);
  if (s->training) {
    const size_t wmax = (size_t)std::max(s->hp, s->out_p);
    A(&s->X0T, Mp * s->in_p0 * s->esz);
    s->HT.assign(s->n_hl, nullptr);
    s->Z.assign(s->n_hl, nullptr);
    for (int l = 0; l < s->n_hl; ++l) {
      A(&s->HT[l], Mp * s->hp * s->esz);
      A(&s->Z[l], Mp * s->hp * s->esz);
    }
    A(&s->dA, Mp * wmax * s->esz);
    A(&s->dAT, Mp * wmax * s->esz);
    A(&s->dB, Mp * wmax * s->esz);
    A(&s->dBT, Mp * wmax * s->esz);
    s->dwp.assign(s->n_layers, nullptr);
    s->dbp.assign(s->n_layers, nullptr);
    for (int l = 0; l < s->n_layers; ++l) {
      A(&s->dwp[l], (size_t)MAX_SLICES * t.out_p[l] * t.in_p[l] * 4);
      A(&s->dbp[l], (Mp / TILE) * t.out_p[l] * 4);
    }
    A(&s->loss_part, (Mp / TILE) * (s->out_p / TILE) * 8);
    A(&s->loss_tmp, 4);
  }
  if (e != hipSuccess) {
    sur_free(s);
    delete s;
    return fail(NPX_ENOMEM, "device allocation for the surrogate failed: %s", hipGetErrorString(e));
  }
  std::vector<float> zero_in(s->n_in, 0.f), one_in(s->n_in, 1.f);
  std::vector<float> zero_out(s->n_out, 0.f), one_out(s->n_out, 1.f);
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  up(s->P, hostP.data(), s->n_pad * 4);
  up(s->x_mean, zero_in.data(), s->n_in * 4);
  up(s->x_inv, one_in.data(), s->n_in * 4);
  up(s->y_mean, zero_out.data(), s->n_out * 4);
  up(s->y_inv, one_out.data(), s->n_out * 4);
  up(s->y_std, one_out.data(), s->n_out * 4);
  if (e == hipSuccess) e = hipMemset(s->G, 0, s->n_pad * 4);
  if (e == hipSuccess) e = hipMemset(s->Mom, 0, s->n_pad * 4);
  if (e == hipSuccess) e = hipMemset(s->Vel, 0, s->n_pad * 4);
  if (e == hipSuccess) e = refresh(s, 0, 0.f, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    sur_free(s);
    delete s;
    return fail(NPX_EHIP, "surrogate initialisation failed: %s", hipGetErrorString(e));
  }
  *out = s;
  return NPX_OK;
}

void npx_sur_destroy(npx_sur* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  sur_free(s);
  delete s;
}

npx_status npx_sur_param_count(const npx_sur* s, int64_t* n) {
  if (!s || !n) return fail(NPX_EINVAL, "null argument");
  *n = s->n_real;
  return NPX_OK;
}

npx_status npx_sur_get_params(npx_sur* s, float* dst, int64_t n, int on_device) {
  if (!s || !dst) return fail(NPX_EINVAL, "null argument");
  if (n != s->n_real) return fail(NPX_EINVAL, "expected %lld parameters", (long long)s->n_real);
  HIP_TRY(hipDeviceSynchronize());
  const int blocks = (int)((s->n_pad + 255) / 256);
  hipLaunchKernelGGL(repack_kernel, dim3(blocks), dim3(256), 0, nullptr, s->tab, 0, s->P, s->flat);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpy(dst, s->flat, n * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  return NPX_OK;
}

npx_status npx_sur_set_params(npx_sur* s, const float* src, int64_t n, int on_device) {
  if (!s || !src) return fail(NPX_EINVAL, "null argument");
  if (n != s->n_real) return fail(NPX_EINVAL, "expected %lld parameters", (long long)s->n_real);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(s->flat, src, n * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
  const int blocks = (int)((s->n_pad + 255) / 256);
  hipLaunchKernelGGL(repack_kernel, dim3(blocks), dim3(256), 0, nullptr, s->tab, 1, s->P, s->flat);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemset(s->Mom, 0, s->n_pad * 4));
  HIP_TRY(hipMemset(s->Vel, 0, s->n_pad * 4));
  s->step = 0;
  HIP_TRY(refresh(s, 0, 0.f, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  return NPX_OK;
}

npx_status npx_sur_set_norm(npx_sur* s, const float* x_mean, const float* x_std,
                            const float* y_mean, const float* y_std) {
  if (!s || !x_mean || !x_std || !y_mean || !y_std) return fail(NPX_EINVAL, "null argument");
  std::vector<float> xi(s->n_in), yi(s->n_out), ys(s->n_out);
  for (int c = 0; c < s->n_in; ++c) {
    if (!(x_std[c] >= 0.f) || !std::isfinite(x_mean[c]))
      return fail(NPX_EINVAL, "input statistics of column %d are not finite", c);
    xi[c] = x_std[c] > 1e-12f ? 1.f / x_std[c] : 1.f;
  }
  for (int c = 0; c < s->n_out; ++c) {
    if (!(y_std[c] >= 0.f) || !std::isfinite(y_mean[c]))
      return fail(NPX_EINVAL, "output statistics of column %d are not finite", c);
    ys[c] = y_std[c] > 1e-12f ? y_std[c] : 1.f;
    yi[c] = 1.f / ys[c];
  }
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(s->x_mean, x_mean, s->n_in * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->x_inv, xi.data(), s->n_in * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->y_mean, y_mean, s->n_out * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->y_inv, yi.data(), s->n_out * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(s->y_std, ys.data(), s->n_out * 4, hipMemcpyHostToDevice));
  return NPX_OK;
}

npx_status npx_sur_set_adam(npx_sur* s, double beta1, double beta2, double eps) {
  if (!s) return fail(NPX_EINVAL, "null surrogate handle");
  if (!(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(NPX_EINVAL, "Adam needs 0 <= beta < 1 and eps > 0");
  s->b1 = beta1;
  s->b2 = beta2;
  s->eps = eps;
  return NPX_OK;
}

npx_status npx_sur_forward(npx_sur* s, const float* x, int64_t ldx, const int32_t* rows,
                           int64_t batch, float* y, int64_t ldy, void* stream) {
  npx_status r = check_io(s, x, ldx, batch);
  if (r != NPX_OK) return r;
  if (batch == 0) return NPX_OK;
  if (!y || ldy < s->n_out) return fail(NPX_EINVAL, "bad output buffer or stride");
  hipStream_t st = (hipStream_t)stream;
  return s->precision == NPX_SUR_FP32
             ? forward_t<float>(s, x, ldx, rows, (int)batch, y, ldy, st)
             : forward_t<__bf16>(s, x, ldx, rows, (int)batch, y, ldy, st);
}

npx_status npx_sur_grad(npx_sur* s, const float* x, int64_t ldx, const float* y, int64_t ldy,
                        const int32_t* rows, int64_t batch, float* loss, float* grad,
                        void* stream) {
  npx_status r = check_io(s, x, ldx, batch);
  if (r != NPX_OK) return r;
  if (!s->training) return fail(NPX_ESTATE, "surrogate was created without training buffers");
  if (batch < 1) return fail(NPX_EINVAL, "empty batch");
  if (!y || ldy < s->n_out) return fail(NPX_EINVAL, "bad target buffer or stride");
  hipStream_t st = (hipStream_t)stream;
  r = s->precision == NPX_SUR_FP32
          ? backward_t<float>(s, x, ldx, y, ldy, rows, (int)batch, loss, st)
          : backward_t<__bf16>(s, x, ldx, y, ldy, rows, (int)batch, loss, st);
  if (r != NPX_OK || !grad) return r;
  const int blocks = (int)((s->n_pad + 255) / 256);
  hipLaunchKernelGGL(repack_kernel, dim3(blocks), dim3(256), 0, st, s->tab, 0, s->G, grad);
  HIP_TRY(hipGetLastError());
  return NPX_OK;
}

npx_status npx_sur_train_step(npx_sur* s, const float* x, int64_t ldx, const float* y,
                              int64_t ldy, const int32_t* rows, int64_t batch, double lr,
                              float* loss, void* stream) {
  if (!(lr >= 0)) return fail(NPX_EINVAL, "learning rate must be >= 0");
  npx_status r = check_io(s, x, ldx, batch);
  if (r != NPX_OK) return r;
  if (!s->training) return fail(NPX_ESTATE, "surrogate was created without training buffers");
  if (batch < 1) return fail(NPX_EINVAL, "empty batch");
  if (!y || ldy < s->n_out) return fail(NPX_EINVAL, "bad target buffer or stride");
  hipStream_t st = (hipStream_t)stream;
  r = s->precision == NPX_SUR_FP32
          ? backward_t<float>(s, x, ldx, y, ldy, rows, (int)batch, loss, st, false)
          : backward_t<__bf16>(s, x, ldx, y, ldy, rows, (int)batch, loss, st, false);
  if (r != NPX_OK) return r;
  s->step += 1;
  const float c1 = (float)(1.0 - std::pow(s->b1, s->step));
  const float c2 = (float)(1.0 - std::pow(s->b2, s->step));
  const int blocks = (int)((s->n_pad + 255) / 256);
  const int n_part = (round_up((int)batch, TILE) / TILE) * (s->out_p / TILE);
  const double inv_count = 1.0 / ((double)batch * s->n_out);
  float* lo = loss ? loss : s->loss_tmp;
  if (s->precision == NPX_SUR_FP32)
    hipLaunchKernelGGL((reduce_adam_kernel<float>), dim3(blocks), dim3(256), 0, st, s->tab, s->G,
                       s->P, s->Mom, s->Vel, (float)lr, (float)s->b1, (float)s->b2, (float)s->eps,
                       c1, c2, static_cast<float*>(s->Wc), static_cast<float*>(s->WTc),
                       s->loss_part, n_part, inv_count, lo);
  else
    hipLaunchKernelGGL((reduce_adam_kernel<__bf16>), dim3(blocks), dim3(256), 0, st, s->tab,
                       s->G, s->P, s->Mom, s->Vel, (float)lr, (float)s->b1, (float)s->b2,
                       (float)s->eps, c1, c2, static_cast<__bf16*>(s->Wc),
                       static_cast<__bf16*>(s->WTc), s->loss_part, n_part, inv_count, lo);
  HIP_TRY(hipGetLastError());
  return NPX_OK;
}

npx_status npx_sur_set_noise(npx_sur* s, const float* noise, int64_t ldn, int32_t col0,
                             int32_t ncols) {
  if (!s) return fail(NPX_EINVAL, "null surrogate handle");
  if (!noise) {
    s->noise = Noise{nullptr, 0, 0, 0};
    return NPX_OK;
  }
  if (col0 < 0 || ncols < 1 || col0 + ncols > s->n_in || col0 + ncols > s->n_out || ldn < ncols)
    return fail(NPX_EINVAL, "noise columns [%d, %d) must lie in both the inputs and the outputs",
                col0, col0 + ncols);
  s->noise = Noise{noise, ldn, col0, ncols};
  return NPX_OK;
}

npx_status npx_sur_norm_stats(const float* x, int64_t ldx, int64_t rows, int32_t cols,
                              float* mean, float* std_out, void* stream) {
  if (!x || !mean || !std_out || rows < 1 || cols < 1 || ldx < cols)
    return fail(NPX_EINVAL, "bad statistics arguments");
  hipStream_t st = (hipStream_t)stream;
  const int64_t chunk = std::max<int64_t>(256, (rows + 1023) / 1024);
  const int nb = (int)((rows + chunk - 1) / chunk);
  double *part = nullptr, *mu = nullptr, *sd = nullptr;
  HIP_TRY(hipMalloc(&part, (size_t)nb * cols * 8));
  hipError_t e = hipMalloc(&mu, (size_t)cols * 8);
  if (e == hipSuccess) e = hipMalloc(&sd, (size_t)cols * 8);
  const int fb = (cols + 255) / 256;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(colstat_kernel, dim3(nb), dim3(256), 0, st, x, ldx, rows, cols, chunk,
                       (const double*)nullptr, 1, part);
    hipLaunchKernelGGL(colstat_final_kernel, dim3(fb), dim3(256), 0, st, part, nb, cols,
                       1.0 / (double)rows, 0, mu, mean);
    hipLaunchKernelGGL(colstat_kernel, dim3(nb), dim3(256), 0, st, x, ldx, rows, cols, chunk,
                       (const double*)mu, 2, part);
    hipLaunchKernelGGL(colstat_final_kernel, dim3(fb), dim3(256), 0, st, part, nb, cols,
                       1.0 / (double)rows, 1, sd, std_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(part);
  if (mu) (void)hipFree(mu);
  if (sd) (void)hipFree(sd);
  if (e != hipSuccess) return fail(NPX_EHIP, "column statistics failed: %s", hipGetErrorString(e));
  return NPX_OK;
}

}  // extern "C"

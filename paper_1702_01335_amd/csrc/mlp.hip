// Warm-start network on gfx950 (C ABI in include/hrlb_mlp.h).
//
// Every matrix product of the forward and backward passes runs through one tiled kernel
// on the matrix cores: 64 x 64 output tiles, four waves of 2 x 2 v_mfma_f32_16x16x32_bf16
// blocks, K steps of 32 staged through LDS.  The operand layouts of that instruction are
// A[m][k] in lane m + 16 (k / 8), element k % 8; B[k][n] in lane n + 16 (k / 8), element
// k % 8; D[4 (l / 16) + r][l % 16] in lane l, result register r (checked on gfx950).
// Operands are addressed through row and column strides, so the three products of a layer
// (Z = H W^T, dH = dZ W, dW = dZ^T H) share the kernel; the epilogue adds the bias and
// applies silu, or multiplies by silu', or stores the fp32 result.  Element-wise work
// (standardisation, loss, bias gradients, AdamW) has kernels of its own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

#include "hrlb_internal.h"
#include "hrlb_mlp.h"

using namespace hrlb;

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int IN = HRLB_MLP_IN, OUT = HRLB_MLP_OUT, WID = HRLB_MLP_WIDTH;
constexpr int K0 = 32;  // input width padded to one K step; the padding columns stay zero
// padded device layout: W0p[256][32] b0 W1 b1 W2 b2 W3[8][256] b3
constexpr int OW0 = 0, OB0 = OW0 + WID * K0, OW1 = OB0 + WID, OB1 = OW1 + WID * WID, OW2 = OB1 + WID,
              OB2 = OW2 + WID * WID, OW3 = OB2 + WID, OB3 = OW3 + OUT * WID, NPAD = OB3 + OUT;
// flat (public) layout: W0[256][5] first, then the same blocks in the same order
constexpr int FB0 = WID * IN, SHIFT = OB0 - FB0;
static_assert(NPAD - SHIFT == HRLB_MLP_NPARAMS, "parameter layouts");
constexpr int NPADR = (NPAD + 63) / 64 * 64;
constexpr int MAX_ROWS = 1 << 22;
constexpr int LOSS_BLOCKS = 1024;
constexpr int LDR = 40;  // LDS row of a 32-wide K step, padded (bf16 elements; 80 bytes)
constexpr int SPLIT_MAX = 16;  // K slices of a split weight-gradient product

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---- device helpers ---------------------------------------------------------------------

// splitmix64 finaliser applied to seed + (i + 1) * golden gamma (Steele, Lea and Flood)
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }

__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// padded index -> flat index, -1 for the zero padding of W0
__device__ __forceinline__ int flat_of(int p) {
  if (p < OB0) {
    const int k = p % K0;
    return k < IN ? (p / K0) * IN + k : -1;
  }
  return p - SHIFT;
}

__device__ __forceinline__ int padded_of(int f) { return f < FB0 ? (f / IN) * K0 + f % IN : f + SHIFT; }

// ---- parameter kernels ------------------------------------------------------------------

__global__ void params_set_kernel(const float* __restrict__ flat, unsigned long long seed, float* master, float* m,
                                  float* v, bf16* wbf) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NPADR; p += gridDim.x * blockDim.x) {
    const int f = p < NPAD ? flat_of(p) : -1;
    float val = 0.0f;
    if (f >= 0) {
      if (flat) {
        val = flat[f];
      } else {
        const int fan_in = f < FB0 + WID ? IN : WID;
        const double u = (double)(splitmix64(seed, (uint64_t)f) >> 11) * 0x1.0p-53;
        val = (float)((2.0 * u - 1.0) / sqrt((double)fan_in));
      }
    }
    master[p] = val;
    m[p] = 0.0f;
    v[p] = 0.0f;
    wbf[p] = (bf16)val;
  }
}

__global__ void params_get_kernel(const float* __restrict__ padded, float* flat) {
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < HRLB_MLP_NPARAMS; f += gridDim.x * blockDim.x)
    flat[f] = padded[padded_of(f)];
}

// AdamW: theta <- theta (1 - lr wd) - lr (m / c1) / (sqrt(v / c2) + eps), then the bf16 copy
__global__ void adamw_kernel(float* master, const float* __restrict__ grad, float* m, float* v, bf16* wbf, float lr,
                             float wd, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NPAD; p += gridDim.x * blockDim.x) {
    const float g = grad[p];
    const float mp = b1 * m[p] + (1.0f - b1) * g;
    const float vp = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mp;
    v[p] = vp;
    float w = master[p] * (1.0f - lr * wd);
    w -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
    master[p] = w;
    wbf[p] = (bf16)w;
  }
}

// ---- row kernels ------------------------------------------------------------------------

// standardised inputs of the selected rows, bf16, padded to K0 columns
__global__ void input_kernel(const float* __restrict__ x, const int* __restrict__ idx, int rows,
                             const float* __restrict__ norm, bf16* x0) {
  const long long total = (long long)rows * K0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / K0), c = (int)(e % K0);
    float val = 0.0f;
    if (c < IN) {
      const long long src = idx ? idx[r] : r;
      val = (x[src * IN + c] - norm[c]) / norm[IN + c];
    }
    x0[e] = (bf16)val;
  }
}

// squared standardised error: dY = bf16(2 (y - t) / (rows * 8)), per-block sums of (y - t)^2
__global__ void __launch_bounds__(256) loss_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                   const int* __restrict__ idx, int rows,
                                                   const float* __restrict__ norm, bf16* dy, float* part) {
  const long long total = (long long)rows * OUT;
  const float scale = 2.0f / (float)total;
  float acc = 0.0f;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / OUT), c = (int)(e % OUT);
    const long long src = idx ? idx[r] : r;
    const float ts = (t[src * OUT + c] - norm[2 * IN + c]) / norm[2 * IN + OUT + c];
    const float d = y[e] - ts;
    dy[e] = (bf16)(scale * d);
    acc += d * d;
  }
  __shared__ float red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) loss_final_kernel(const float* __restrict__ part, int nblk, int rows,
                                                         float* loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(red[0] / ((double)rows * OUT));
}

// bias gradient: column sums of dZ[rows][n].  Block (x, y) sums 64 columns over the y-th
// slice of rows (4 row phases, then a fixed-order LDS sum) into part[y][n]; a second
// kernel adds the slices in order.
__global__ void __launch_bounds__(256) colsum_kernel(const bf16* __restrict__ dz, int rows, int n, int slice,
                                                     float* part) {
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  const int r0 = blockIdx.y * slice, r1 = min(rows, r0 + slice);
  float s = 0.0f;
  if (c < n)
    for (int r = r0 + g; r < r1; r += 4) s += (float)dz[(size_t)r * n + c];
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && c < n)
    part[(size_t)blockIdx.y * n + c] =
        ((red[threadIdx.x] + red[threadIdx.x + 64]) + red[threadIdx.x + 128]) + red[threadIdx.x + 192];
}

__global__ void colsum_reduce_kernel(const float* __restrict__ part, int nslices, int n, float* db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float s = 0.0f;
  for (int y = 0; y < nslices; ++y) s += part[(size_t)y * n + c];
  db[c] = s;
}

hipError_t colsum(const bf16* dz, int rows, int n, float* ws, float* db, hipStream_t st) {
  // at most 256 slices, so the partials fit the split-K workspace (256 x n <= SPLIT_MAX x 256 x 256)
  const int slice = std::max(64, (rows + 255) / 256), ns = (rows + slice - 1) / slice;
  hipLaunchKernelGGL(colsum_kernel, dim3((n + 63) / 64, ns), dim3(256), 0, st, dz, rows, n, slice, ws);
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, st, ws, ns, n, db);
  return hipGetLastError();
}

// raw outputs y * std + mean, as fp32 rows or as an fp64 Couette moment table
__global__ void output_kernel(const float* __restrict__ y, int rows, const float* __restrict__ norm, float* out,
                              double* table) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x) {
    float o[OUT];
#pragma unroll
    for (int c = 0; c < OUT; ++c) o[c] = y[(size_t)r * OUT + c] * norm[2 * IN + OUT + c] + norm[2 * IN + c];
    if (out) {
#pragma unroll
      for (int c = 0; c < OUT; ++c) out[(size_t)r * OUT + c] = o[c];
    }
    if (table) {
      // channels n, u_y, T, P_xx, P_xy, P_yy, q_x, q_y -> n ux uy uz T Pxx Pyy Pzz Pxy Pxz Pyz qx qy qz
      const double n = o[0], T = o[2], Pxx = o[3], Pyy = o[5];
      double* tr = table + (size_t)r * 14;
      tr[0] = n;
      tr[1] = 0.0;
      tr[2] = o[1];
      tr[3] = 0.0;
      tr[4] = T;
      tr[5] = Pxx;
      tr[6] = Pyy;
      tr[7] = 3.0 * n * T - Pxx - Pyy;
      tr[8] = o[4];
      tr[9] = 0.0;
      tr[10] = 0.0;
      tr[11] = o[6];
      tr[12] = o[7];
      tr[13] = 0.0;
    }
  }
}

// ---- matrix product on the matrix cores ------------------------------------------------

enum { EPI_HIDDEN = 0, EPI_OUTPUT = 1, EPI_DSILU = 2, EPI_STORE = 3 };

struct Gemm {
  const bf16* A;
  long long sar, sac;  // A(i, k) = A[i sar + k sac], i < M, k < K
  const bf16* B;
  long long sbk, sbj;  // B(k, j) = B[k sbk + j sbj], j < N
  int M, N, K;
  const float* bias;   // EPI_HIDDEN, EPI_OUTPUT: bias[j]
  const float* zin;    // EPI_DSILU: pre-activation zin[i ldz + j]
  int ldz;
  float* C;            // EPI_HIDDEN (z), EPI_OUTPUT, EPI_STORE: C[i ldc + j]
  int ldc;
  bf16* H;             // EPI_HIDDEN (silu z), EPI_DSILU (dz): H[i ldh + j]
  int ldh;
  int kc;              // K values per slice (set by the launcher)
  float* part;         // split-K partial products [slices][M][N], or NULL
};

// One 64 x 32 operand tile (64 rows of the operand, 32 K values) into LDS as [row][k],
// zero beyond the matrix.  Two access patterns, chosen per launch: with K contiguous each
// thread loads 8 consecutive K values of one row; with rows contiguous (a transposed
// operand) each thread loads 8 consecutive rows at one K value and scatters them.
// 16-byte vector loads where the whole vector is inside the matrix and aligned.
__device__ __forceinline__ void stage_tile(const bf16* __restrict__ base, long long srow, long long sk, int row0,
                                           int nrows, int k0, int K, bf16* lds) {
  const int tid = threadIdx.x;
  if (sk == 1 || srow != 1) {
    const int r = tid >> 2, kc = (tid & 3) * 8, row = row0 + r, k = k0 + kc;
    bf16* dst = lds + r * LDR + kc;
    const bool row_ok = row < nrows;
    const bf16* src = base + (row_ok ? (long long)row * srow : 0);
    if (row_ok && sk == 1 && k + 8 <= K && ((((uintptr_t)(src + k)) & 15) == 0)) {
      *(bf16x8*)dst = *(const bf16x8*)(src + k);
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) dst[e] = (row_ok && k + e < K) ? src[(long long)(k + e) * sk] : (bf16)0.0f;
  } else {
    const int kk = tid >> 3, rc = (tid & 7) * 8, k = k0 + kk, row = row0 + rc;
    bf16* dst = lds + rc * LDR + kk;
    const bool k_ok = k < K;
    const bf16* src = base + (k_ok ? (long long)k * sk : 0);
    if (k_ok && row + 8 <= nrows && ((((uintptr_t)(src + row)) & 15) == 0)) {
      const bf16x8 v = *(const bf16x8*)(src + row);
#pragma unroll
      for (int e = 0; e < 8; ++e) dst[e * LDR] = v[e];
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) dst[e * LDR] = (k_ok && row + e < nrows) ? src[row + e] : (bf16)0.0f;
  }
}

// blockIdx.z selects a slice of K of kc values (a multiple of 32); with more than one slice
// the raw products go to part[z][M][N] and a second kernel adds the slices in order.
template <int EPI>
__global__ void __launch_bounds__(256) gemm_kernel(Gemm g) {
  __shared__ __attribute__((aligned(16))) bf16 As[64 * LDR];
  __shared__ __attribute__((aligned(16))) bf16 Bs[64 * LDR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int kbeg = blockIdx.z * g.kc, kend = min(g.K, kbeg + g.kc);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
    stage_tile(g.A, g.sar, g.sac, i0, g.M, k0, kend, As);
    stage_tile(g.B, g.sbj, g.sbk, j0, g.N, k0, kend, Bs);
    __syncthreads();
    const bf16x8 a0 = *(const bf16x8*)&As[(wm + fr) * LDR + fk];
    const bf16x8 a1 = *(const bf16x8*)&As[(wm + 16 + fr) * LDR + fk];
    const bf16x8 b0 = *(const bf16x8*)&Bs[(wn + fr) * LDR + fk];
    const bf16x8 b1 = *(const bf16x8*)&Bs[(wn + 16 + fr) * LDR + fk];
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
    __syncthreads();
  }
  float* part = g.part ? g.part + (size_t)blockIdx.z * g.M * g.N : nullptr;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm + 16 * bi + 4 * (lane >> 4) + r;
        const int j = j0 + wn + 16 * bj + (lane & 15);
        if (i >= g.M || j >= g.N) continue;
        const float v = acc[bi][bj][r];
        if (EPI == EPI_HIDDEN) {
          const float z = v + g.bias[j];
          g.C[(size_t)i * g.ldc + j] = z;
          g.H[(size_t)i * g.ldh + j] = (bf16)silu(z);
        } else if (EPI == EPI_OUTPUT) {
          g.C[(size_t)i * g.ldc + j] = v + g.bias[j];
        } else if (EPI == EPI_DSILU) {
          g.H[(size_t)i * g.ldh + j] = (bf16)(v * silu_grad(g.zin[(size_t)i * g.ldz + j]));
        } else if (part) {
          part[(size_t)i * g.N + j] = v;
        } else {
          g.C[(size_t)i * g.ldc + j] = v;
        }
      }
}

// C[i][j] = sum over slices z (in order) of part[z][i][j]
__global__ void splitk_reduce_kernel(const float* __restrict__ part, int nz, int M, int N, float* C, int ldc) {
  const int total = M * N;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int z = 0; z < nz; ++z) s += part[(size_t)z * total + e];
    C[(size_t)(e / N) * ldc + e % N] = s;
  }
}

template <int EPI>
hipError_t gemm(Gemm g, hipStream_t st, float* split_ws = nullptr) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  int nz = 1;
  // long reductions over few output tiles (the weight gradients): split K so the grid
  // fills the chip; the slices are added by a second kernel in a fixed order
  const int tiles = ((g.N + 63) / 64) * ((g.M + 63) / 64);
  if (EPI == EPI_STORE && split_ws && tiles < 256 && g.K > 512) {
    nz = std::min(SPLIT_MAX, std::max(1, 256 / tiles));
    nz = std::min(nz, (g.K + 255) / 256);
  }
  g.kc = ((g.K + nz - 1) / nz + 31) / 32 * 32;
  nz = (g.K + g.kc - 1) / g.kc;
  g.part = nz > 1 ? split_ws : nullptr;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, nz);
  hipLaunchKernelGGL(gemm_kernel<EPI>, grid, dim3(256), 0, st, g);
  if (nz > 1)
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(std::min(1024, (g.M * g.N + 255) / 256)), dim3(256), 0, st, split_ws,
                       nz, g.M, g.N, g.C, g.ldc);
  return hipGetLastError();
}

Gemm make(const bf16* A, long long sar, long long sac, const bf16* B, long long sbk, long long sbj, int M, int N,
          int K) {
  Gemm g;
  std::memset(&g, 0, sizeof(g));
  g.A = A;
  g.sar = sar;
  g.sac = sac;
  g.B = B;
  g.sbk = sbk;
  g.sbj = sbj;
  g.M = M;
  g.N = N;
  g.K = K;
  return g;
}

int grid_for(long long n) { return (int)std::min<long long>((n + 255) / 256, 4096); }

}  // namespace

struct hrlb_mlp {
  float* master;
  float* m;
  float* v;
  bf16* wbf;
  float* norm;
  bf16* x0;
  float* z[3];
  bf16* h[3];
  float* y;
  bf16* dy;
  bf16* dz[2];
  float* grad;
  float* part;
  float* loss;
  float* split;
  int max_rows;
  long long t;
  hipStream_t stream;
};

namespace {

size_t state_bytes_of() { return 3 * a256((size_t)NPADR * 4) + a256((size_t)NPADR * 2) + 256; }

size_t work_bytes_of(int rows) {
  const size_t Mp = ((size_t)rows + 63) / 64 * 64;
  return a256(Mp * K0 * 2) + 3 * a256(Mp * WID * 4) + 3 * a256(Mp * WID * 2) + a256(Mp * OUT * 4) +
         a256(Mp * OUT * 2) + 2 * a256(Mp * WID * 2) + a256((size_t)NPADR * 4) + a256(LOSS_BLOCKS * 4) + 256 +
         a256((size_t)SPLIT_MAX * WID * WID * 4);
}

hipError_t set_norm(hrlb_mlp* m, const float* h_norm) {
  float buf[64] = {0};
  std::memcpy(buf, h_norm, HRLB_MLP_NORM * sizeof(float));
  hipError_t e = hipMemcpyAsync(m->norm, buf, 64 * sizeof(float), hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  return e;
}

bool norm_ok(const float* h) {
  for (int i = 0; i < HRLB_MLP_NORM; ++i)
    if (!std::isfinite(h[i])) return false;
  for (int i = 0; i < IN; ++i)
    if (!(h[IN + i] > 0.0f)) return false;
  for (int i = 0; i < OUT; ++i)
    if (!(h[2 * IN + OUT + i] > 0.0f)) return false;
  return true;
}

// forward pass of the selected rows; leaves standardised outputs in m->y
hipError_t forward(hrlb_mlp* m, const float* x, const int* idx, int rows) {
  hipStream_t st = m->stream;
  hipLaunchKernelGGL(input_kernel, dim3(grid_for((long long)rows * K0)), dim3(256), 0, st, x, idx, rows, m->norm, m->x0);
  hipError_t e = hipGetLastError();
  const bf16* hin = m->x0;
  int kin = K0;
  const int ow[3] = {OW0, OW1, OW2}, ob[3] = {OB0, OB1, OB2};
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    Gemm g = make(hin, kin, 1, m->wbf + ow[l], 1, kin, rows, WID, kin);
    g.bias = m->master + ob[l];
    g.C = m->z[l];
    g.ldc = WID;
    g.H = m->h[l];
    g.ldh = WID;
    e = gemm<EPI_HIDDEN>(g, st);
    hin = m->h[l];
    kin = WID;
  }
  if (e == hipSuccess) {
    Gemm g = make(m->h[2], WID, 1, m->wbf + OW3, 1, WID, rows, OUT, WID);
    g.bias = m->master + OB3;
    g.C = m->y;
    g.ldc = OUT;
    e = gemm<EPI_OUTPUT>(g, st);
  }
  return e;
}

// loss, then the gradient of every parameter into m->grad (padded layout)
hipError_t backward(hrlb_mlp* m, const float* t, const int* idx, int rows, float* loss_out) {
  hipStream_t st = m->stream;
  const int nblk = std::min(LOSS_BLOCKS, grid_for((long long)rows * OUT));
  hipLaunchKernelGGL(loss_kernel, dim3(nblk), dim3(256), 0, st, m->y, t, idx, rows, m->norm, m->dy, m->part);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, m->part, nblk, rows,
                     loss_out ? loss_out : m->loss);
  hipError_t e = hipGetLastError();
  // output layer: dW3 = dY^T H2, db3 = colsum dY, dZ2 = (dY W3) * silu'(Z2)
  {
    Gemm g = make(m->dy, 1, OUT, m->h[2], WID, 1, OUT, WID, rows);
    g.C = m->grad + OW3;
    g.ldc = WID;
    if (e == hipSuccess) e = gemm<EPI_STORE>(g, st, m->split);
    if (e == hipSuccess) e = colsum(m->dy, rows, OUT, m->split, m->grad + OB3, st);
    Gemm d = make(m->dy, OUT, 1, m->wbf + OW3, WID, 1, rows, WID, OUT);
    d.zin = m->z[2];
    d.ldz = WID;
    d.H = m->dz[0];
    d.ldh = WID;
    if (e == hipSuccess) e = gemm<EPI_DSILU>(d, st);
  }
  const int ow[3] = {OW0, OW1, OW2}, ob[3] = {OB0, OB1, OB2};
  int cur = 0;
  for (int l = 2; l >= 0 && e == hipSuccess; --l) {
    const bf16* hin = l > 0 ? m->h[l - 1] : m->x0;
    const int kin = l > 0 ? WID : K0;
    const bf16* dz = m->dz[cur];
    Gemm g = make(dz, 1, WID, hin, kin, 1, WID, kin, rows);
    g.C = m->grad + ow[l];
    g.ldc = kin;
    e = gemm<EPI_STORE>(g, st, m->split);
    if (e == hipSuccess) e = colsum(dz, rows, WID, m->split, m->grad + ob[l], st);
    if (l > 0 && e == hipSuccess) {
      Gemm d = make(dz, WID, 1, m->wbf + ow[l], kin, 1, rows, WID, WID);
      d.zin = m->z[l - 1];
      d.ldz = WID;
      d.H = m->dz[1 - cur];
      d.ldh = WID;
      e = gemm<EPI_DSILU>(d, st);
      cur = 1 - cur;
    }
  }
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}

int check_rows(const hrlb_mlp* m, const float* x, int rows) {
  if (!m || !x) return set_error(HRLB_EINVAL, "mlp: NULL argument");
  if (rows < 1 || rows > m->max_rows) return set_error(HRLB_EINVAL, "mlp: rows must be in 1..max_rows");
  return HRLB_OK;
}

}  // namespace

extern "C" {

int hrlb_mlp_bytes(int max_rows, size_t* state_bytes, size_t* work_bytes) {
  if (!state_bytes || !work_bytes) return set_error(HRLB_EINVAL, "mlp_bytes: NULL argument");
  if (max_rows < 1 || max_rows > MAX_ROWS) return set_error(HRLB_EINVAL, "mlp_bytes: max_rows must be in 1..2^22");
  *state_bytes = state_bytes_of();
  *work_bytes = work_bytes_of(max_rows);
  return HRLB_OK;
}

int hrlb_mlp_create(void* d_state, size_t state_bytes, void* d_work, size_t work_bytes, int max_rows,
                    const float* d_params, unsigned long long seed, const float* h_norm, void* stream,
                    hrlb_mlp** out) {
  if (!out) return set_error(HRLB_EINVAL, "mlp_create: out is NULL");
  *out = nullptr;
  if (!d_state || !d_work || !h_norm) return set_error(HRLB_EINVAL, "mlp_create: NULL argument");
  if (((uintptr_t)d_state & 255) || ((uintptr_t)d_work & 255))
    return set_error(HRLB_EINVAL, "mlp_create: buffers must be 256-byte aligned");
  if (max_rows < 1 || max_rows > MAX_ROWS) return set_error(HRLB_EINVAL, "mlp_create: max_rows must be in 1..2^22");
  if (state_bytes < state_bytes_of() || work_bytes < work_bytes_of(max_rows))
    return set_error(HRLB_ENOMEM, "mlp_create: buffer smaller than hrlb_mlp_bytes requires");
  if (!norm_ok(h_norm)) return set_error(HRLB_EINVAL, "mlp_create: standardisation constants not finite or std <= 0");
  hrlb_mlp* m = new hrlb_mlp;
  std::memset(m, 0, sizeof(*m));
  m->stream = (hipStream_t)stream;
  m->max_rows = max_rows;
  char* s = (char*)d_state;
  m->master = (float*)s;
  s += a256((size_t)NPADR * 4);
  m->m = (float*)s;
  s += a256((size_t)NPADR * 4);
  m->v = (float*)s;
  s += a256((size_t)NPADR * 4);
  m->wbf = (bf16*)s;
  s += a256((size_t)NPADR * 2);
  m->norm = (float*)s;
  const size_t Mp = ((size_t)max_rows + 63) / 64 * 64;
  char* w = (char*)d_work;
  m->x0 = (bf16*)w;
  w += a256(Mp * K0 * 2);
  for (int l = 0; l < 3; ++l) {
    m->z[l] = (float*)w;
    w += a256(Mp * WID * 4);
  }
  for (int l = 0; l < 3; ++l) {
    m->h[l] = (bf16*)w;
    w += a256(Mp * WID * 2);
  }
  m->y = (float*)w;
  w += a256(Mp * OUT * 4);
  m->dy = (bf16*)w;
  w += a256(Mp * OUT * 2);
  for (int l = 0; l < 2; ++l) {
    m->dz[l] = (bf16*)w;
    w += a256(Mp * WID * 2);
  }
  m->grad = (float*)w;
  w += a256((size_t)NPADR * 4);
  m->part = (float*)w;
  w += a256(LOSS_BLOCKS * 4);
  m->loss = (float*)w;
  w += 256;
  m->split = (float*)w;
  hipError_t e = set_norm(m, h_norm);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(params_set_kernel, dim3(grid_for(NPADR)), dim3(256), 0, m->stream, d_params, seed, m->master,
                       m->m, m->v, m->wbf);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    // the padded gradient entries are never written by the products: clear them once
    e = hipMemsetAsync(m->grad, 0, (size_t)NPADR * 4, m->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    delete m;
    return set_error(HRLB_EHIP, (std::string("mlp_create: ") + hipGetErrorString(e)).c_str());
  }
  *out = m;
  return HRLB_OK;
}

int hrlb_mlp_set_params(hrlb_mlp* m, const float* d_params) {
  if (!m || !d_params) return set_error(HRLB_EINVAL, "mlp_set_params: NULL argument");
  hipLaunchKernelGGL(params_set_kernel, dim3(grid_for(NPADR)), dim3(256), 0, m->stream, d_params, 0ull, m->master,
                     m->m, m->v, m->wbf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(HRLB_EHIP, hipGetErrorString(e));
  m->t = 0;
  return HRLB_OK;
}

int hrlb_mlp_get_params(hrlb_mlp* m, float* d_params) {
  if (!m || !d_params) return set_error(HRLB_EINVAL, "mlp_get_params: NULL argument");
  hipLaunchKernelGGL(params_get_kernel, dim3(grid_for(HRLB_MLP_NPARAMS)), dim3(256), 0, m->stream, m->master, d_params);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HRLB_OK : set_error(HRLB_EHIP, hipGetErrorString(e));
}

int hrlb_mlp_forward(hrlb_mlp* m, const float* d_x, int rows, float* d_y) {
  int rc = check_rows(m, d_x, rows);
  if (rc != HRLB_OK) return rc;
  if (!d_y) return set_error(HRLB_EINVAL, "mlp_forward: NULL output");
  hipError_t e = forward(m, d_x, nullptr, rows);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(output_kernel, dim3(grid_for(rows)), dim3(256), 0, m->stream, m->y, rows, m->norm, d_y,
                       (double*)nullptr);
    e = hipGetLastError();
  }
  return e == hipSuccess ? HRLB_OK : set_error(HRLB_EHIP, hipGetErrorString(e));
}

int hrlb_mlp_predict_table(hrlb_mlp* m, const float* d_x, int rows, double* d_table) {
  int rc = check_rows(m, d_x, rows);
  if (rc != HRLB_OK) return rc;
  if (!d_table) return set_error(HRLB_EINVAL, "mlp_predict_table: NULL output");
  hipError_t e = forward(m, d_x, nullptr, rows);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(output_kernel, dim3(grid_for(rows)), dim3(256), 0, m->stream, m->y, rows, m->norm,
                       (float*)nullptr, d_table);
    e = hipGetLastError();
  }
  return e == hipSuccess ? HRLB_OK : set_error(HRLB_EHIP, hipGetErrorString(e));
}

int hrlb_mlp_gradient(hrlb_mlp* m, const float* d_x, const float* d_t, const int* d_idx, int rows, float* d_grad,
                      float* d_loss) {
  int rc = check_rows(m, d_x, rows);
  if (rc != HRLB_OK) return rc;
  if (!d_t || !d_grad) return set_error(HRLB_EINVAL, "mlp_gradient: NULL argument");
  hipError_t e = forward(m, d_x, d_idx, rows);
  if (e == hipSuccess) e = backward(m, d_t, d_idx, rows, d_loss);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(params_get_kernel, dim3(grid_for(HRLB_MLP_NPARAMS)), dim3(256), 0, m->stream, m->grad, d_grad);
    e = hipGetLastError();
  }
  return e == hipSuccess ? HRLB_OK : set_error(HRLB_EHIP, hipGetErrorString(e));
}

int hrlb_mlp_train_step(hrlb_mlp* m, const float* d_x, const float* d_t, const int* d_idx, int rows, float lr,
                        float wd, float* d_loss) {
  int rc = check_rows(m, d_x, rows);
  if (rc != HRLB_OK) return rc;
  if (!d_t) return set_error(HRLB_EINVAL, "mlp_train_step: NULL targets");
  if (!(lr > 0.0f) || !(wd >= 0.0f)) return set_error(HRLB_EINVAL, "mlp_train_step: need lr > 0 and wd >= 0");
  hipError_t e = forward(m, d_x, d_idx, rows);
  if (e == hipSuccess) e = backward(m, d_t, d_idx, rows, d_loss);
  if (e == hipSuccess) {
    m->t += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)m->t));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)m->t));
    hipLaunchKernelGGL(adamw_kernel, dim3(grid_for(NPAD)), dim3(256), 0, m->stream, m->master, m->grad, m->m, m->v,
                       m->wbf, lr, wd, c1, c2);
    e = hipGetLastError();
  }
  return e == hipSuccess ? HRLB_OK : set_error(HRLB_EHIP, hipGetErrorString(e));
}

void hrlb_mlp_free(hrlb_mlp* m) { delete m; }

}  // extern "C"

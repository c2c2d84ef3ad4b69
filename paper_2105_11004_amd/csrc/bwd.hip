// Adjoint of f(A) = sum_i w_i theta~_i with the sketch (S, G, G_k), the
// pivots K and the rank r held fixed.  With Y = A_K Z = A Z_full:
//
//   C      = A^T diag(w) A Z_full          (d x k; rows by column id)
//   Zbar   = 2 C[K, :]                      (small FP64 core, host-ordered
//   ...    -> H = G^T (QR adjoint)           launches in lev_api.cpp)
//   Abar_i = 2 w_i Y_i Z_full^T + s_i H_full[h(i), :]
//
// Two passes over A run here: bwd_gram (C) and bwd_grad (Abar).  Both stage
// 64-row (or 32/16-row) tiles of A in LDS and contract them on the matrix
// cores with 16x16x4 MFMAs (FP32 for FP32 A, FP64 for FP64 A); Y is
// recomputed in each pass rather than stored.  The gradient is not part of
// the paper; it makes the estimator usable inside a differentiable program.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lev_device.h"
#include "lev_internal.h"

namespace lev {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA: operand A lane l = A[l % 16][l / 16], operand B lane l =
// B[l / 16][l % 16]; the accumulator's element v of lane l is row row(l, v),
// column l % 16 (the FP32 and FP64 instructions order rows differently).
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  using Acc = v4f;
  __device__ static Acc run(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <>
struct Mfma<double> {
  using Acc = v4d;
  __device__ static Acc run(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int v) { return (l >> 4) + 4 * v; }
};

constexpr int kThreads = 256;
constexpr int kWaves = 4;
constexpr int kZCols = 64;       // Z_full row length in global memory (k padded)
constexpr int kMaxCBlocks = 12;  // C blocks (16 x 16) held per wave in bwd_gram

// Row strides in LDS, in elements, padded so that the MFMA operand reads
// spread over the banks.
template <typename T>
__host__ __device__ constexpr int pad_stride(int cols) {
  return cols + (sizeof(T) == 4 ? 4 : 2);
}

struct TileGeom {
  int TM;   // rows per tile (64, 32 or 16)
  int d16;  // d rounded up to 16
  int kb;   // 16-column blocks of k
  int sa, sz, sy;  // LDS strides of the A tile, of Z_full and of Y
};

template <typename T>
__host__ TileGeom tile_geom(int64_t d, int64_t k) {
  TileGeom g;
  g.d16 = (int)((d + 15) / 16 * 16);
  g.kb = (int)((k + 15) / 16);
  g.sa = pad_stride<T>(g.d16);
  g.sz = pad_stride<T>(16 * g.kb);
  g.sy = pad_stride<T>(16 * g.kb);
  g.TM = 64;
  while (g.TM > 16 && (size_t)g.TM * g.sa * sizeof(T) > 72 * 1024) g.TM /= 2;
  return g;
}

template <typename T>
__host__ size_t lds_bytes(const TileGeom& g, bool zlds) {
  size_t b = (size_t)g.TM * g.sa * sizeof(T) + (size_t)g.TM * g.sy * sizeof(T) + 2 * g.TM * sizeof(int32_t);
  if (zlds) b += (size_t)g.d16 * g.sz * sizeof(T);
  return b;
}

// Cooperative load of rows [r0, r0 + TM) of A into As (zero past n and d).
// Row starts are 16-byte aligned (the interface requires it), so whole
// 16-byte vectors are read; the vector holding column d-1 is masked.
template <typename T>
__device__ void load_tile(const T* __restrict__ A, int64_t n, int64_t d, int64_t ld, int64_t r0,
                          const TileGeom& g, T* As) {
  constexpr int E = 16 / sizeof(T);
  const int vec_per_row = g.d16 / E;
  const int total = g.TM * vec_per_row;
  for (int q = threadIdx.x; q < total; q += kThreads) {
    const int row = q / vec_per_row;
    const int c0 = (q % vec_per_row) * E;
    const int64_t i = r0 + row;
    T v[E];
    if (i < n && c0 < d) {
      const uint4 raw = *reinterpret_cast<const uint4*>(A + i * ld + c0);
      __builtin_memcpy(v, &raw, 16);
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (c0 + e >= d) v[e] = 0;
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = 0;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) As[row * g.sa + c0 + e] = v[e];
  }
}

// Y (TM x 16 kb) = A_tile Z_full, times scale * w_i, into Ys.  Block b of
// the (TM/16) x kb grid of 16 x 16 blocks goes to wave b % 4.
template <typename T, bool ZLDS>
__device__ void tile_y(const T* As, const T* Zs, const T* __restrict__ Zg, int64_t n_zrows, const T* __restrict__ w,
                       int64_t n, int64_t r0, T scale, const TileGeom& g, T* Ys) {
  using M = Mfma<T>;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nblk = (g.TM / 16) * g.kb;
  for (int b = wave; b < nblk; b += kWaves) {
    const int mb = b / g.kb, nb = b % g.kb;
    typename M::Acc acc = {0, 0, 0, 0};
    const T* arow = As + (16 * mb + (lane & 15)) * g.sa + (lane >> 4);
    for (int s = 0; s < g.d16 / 4; ++s) {
      const T a = arow[4 * s];
      const int zr = 4 * s + (lane >> 4), zc = 16 * nb + (lane & 15);
      const T z = ZLDS ? Zs[zr * g.sz + zc] : (zr < n_zrows ? Zg[(int64_t)zr * kZCols + zc] : (T)0);
      acc = M::run(a, z, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * mb + M::row(lane, v);
      const int64_t i = r0 + row;
      const T wi = i < n ? (w != nullptr ? w[i] : (T)1) : (T)0;  // w = null: all ones
      Ys[row * g.sy + 16 * nb + (lane & 15)] = acc[v] * wi * scale;
    }
  }
}

template <typename T, bool ZLDS>
__device__ void stage_z(const T* __restrict__ Zg, int64_t d, const TileGeom& g, T* Zs) {
  if (!ZLDS) return;
  const int cols = 16 * g.kb;
  for (int q = threadIdx.x; q < g.d16 * cols; q += kThreads) {
    const int r = q / cols, c = q % cols;
    Zs[r * g.sz + c] = r < d ? Zg[(int64_t)r * kZCols + c] : (T)0;
  }
}

// C partial of this workgroup (d x 64, rows >= d and columns >= 16 kb left
// untouched) = sum over its tiles of A_tile^T (w o Y_tile).  The (d16/16) x
// kb blocks of C are split over grid.y slices; within a slice block j goes to
// wave j % 4 and stays in its registers for the whole pass.
template <typename T, bool ZLDS>
__global__ __launch_bounds__(kThreads) void bwd_gram_kernel(const T* __restrict__ A, int64_t n, int64_t d, int64_t ld,
                                                            const T* __restrict__ w, const T* __restrict__ Zg,
                                                            TileGeom g, int blocks_per_slice,
                                                            T* __restrict__ partials) {
  using M = Mfma<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = reinterpret_cast<T*>(smem);
  T* Ys = As + g.TM * g.sa;
  T* Zs = Ys + g.TM * g.sy + (2 * g.TM * sizeof(int32_t) + sizeof(T) - 1) / sizeof(T);
  stage_z<T, ZLDS>(Zg, d, g, Zs);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int total_blocks = (g.d16 / 16) * g.kb;
  const int first = blockIdx.y * blocks_per_slice;
  const int last = std::min(total_blocks, first + blocks_per_slice);
  typename M::Acc acc[kMaxCBlocks];
#pragma unroll
  for (int j = 0; j < kMaxCBlocks; ++j) acc[j] = typename M::Acc{0, 0, 0, 0};

  const int64_t ntiles = (n + g.TM - 1) / g.TM;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * g.TM;
    __syncthreads();  // previous tile's readers are done with As and Ys
    load_tile<T>(A, n, d, ld, r0, g, As);
    __syncthreads();
    tile_y<T, ZLDS>(As, Zs, Zg, d, w, n, r0, (T)1, g, Ys);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kMaxCBlocks; ++j) {
      const int b = first + wave + kWaves * j;
      if (b < last) {
        const int db = b / g.kb, nb = b % g.kb;
        const T* ap = As + (lane >> 4) * g.sa + 16 * db + (lane & 15);
        const T* yp = Ys + (lane >> 4) * g.sy + 16 * nb + (lane & 15);
        for (int s = 0; s < g.TM / 4; ++s) acc[j] = M::run(ap[4 * s * g.sa], yp[4 * s * g.sy], acc[j]);
      }
    }
  }
  T* out = partials + (int64_t)blockIdx.x * d * kZCols;
#pragma unroll
  for (int j = 0; j < kMaxCBlocks; ++j) {
    const int b = first + wave + kWaves * j;
    if (b < last) {
      const int db = b / g.kb, nb = b % g.kb;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * db + M::row(lane, v);
        if (row < d) out[(int64_t)row * kZCols + 16 * nb + (lane & 15)] = acc[j][v];
      }
    }
  }
}

// C64[i][c] = sum over workgroups g (ascending) of partials[g][i][c].
template <typename T>
__global__ void bwd_reduce_kernel(const T* __restrict__ partials, int groups, int64_t d, int64_t k,
                                  double* __restrict__ C64) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * k) return;
  const int64_t i = idx / k, c = idx % k;
  const T* p = partials + i * kZCols + c;
  const int64_t step = d * kZCols;
  double s = 0.0;
  // sixteen loads in flight at a time; the sum stays in group order
  int q = 0;
  for (; q + 16 <= groups; q += 16) {
    T v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = p[(int64_t)(q + u) * step];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += (double)v[u];
  }
  for (; q < groups; ++q) s += (double)p[(int64_t)q * step];
  C64[idx] = s;
}

// Abar rows of the tile: 2 w_i Y_i Z_full^T + s_i H_full[h(i), :].
template <typename T, bool ZLDS>
__global__ __launch_bounds__(kThreads) void bwd_grad_kernel(const T* __restrict__ A, int64_t n, int64_t d, int64_t ld,
                                                            const T* __restrict__ w, const T* __restrict__ Zg,
                                                            const T* __restrict__ Hf, HashParams hp, TileGeom g,
                                                            T* __restrict__ G, int64_t ldg) {
  using M = Mfma<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = reinterpret_cast<T*>(smem);
  T* Ys = As + g.TM * g.sa;
  int32_t* hrow = reinterpret_cast<int32_t*>(Ys + g.TM * g.sy);
  int32_t* srow = hrow + g.TM;
  T* Zs = Ys + g.TM * g.sy + (2 * g.TM * sizeof(int32_t) + sizeof(T) - 1) / sizeof(T);
  stage_z<T, ZLDS>(Zg, d, g, Zs);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t ntiles = (n + g.TM - 1) / g.TM;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * g.TM;
    __syncthreads();
    load_tile<T>(A, n, d, ld, r0, g, As);
    for (int q = threadIdx.x; q < g.TM; q += kThreads) {
      const int64_t i = r0 + q;
      if (i < n) {
        const uint64_t x = hash_x(hp, (uint64_t)i);
        hrow[q] = (int32_t)((uint32_t)x % (uint32_t)hp.r_cs);  // x < P < 2^32
        srow[q] = sign_negative(hp, (uint64_t)i) ? -1 : 1;
      } else {
        hrow[q] = 0;
        srow[q] = 0;
      }
    }
    __syncthreads();
    tile_y<T, ZLDS>(As, Zs, Zg, d, w, n, r0, (T)2, g, Ys);
    __syncthreads();
    const int nblk = (g.TM / 16) * (g.d16 / 16);
    for (int b = wave; b < nblk; b += kWaves) {
      const int mb = b % (g.TM / 16), db = b / (g.TM / 16);
      typename M::Acc acc = {0, 0, 0, 0};
      const T* yp = Ys + (16 * mb + (lane & 15)) * g.sy + (lane >> 4);
      const int zrow = 16 * db + (lane & 15);
      for (int s = 0; s < 4 * g.kb; ++s) {
        const int zc = 4 * s + (lane >> 4);
        const T z = ZLDS ? Zs[zrow * g.sz + zc] : (zrow < d ? Zg[(int64_t)zrow * kZCols + zc] : (T)0);
        acc = M::run(yp[4 * s], z, acc);
      }
      const int col = 16 * db + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * mb + M::row(lane, v);
        const int64_t i = r0 + row;
        if (i < n && col < d) {
          const T hv = Hf[(int64_t)hrow[row] * d + col];
          G[i * ldg + col] = acc[v] + (srow[row] < 0 ? -hv : hv);
        }
      }
    }
  }
}

// Abar for FP32 A with d a multiple of 16 (d <= 256) and k <= 64, without
// staging A: each wave owns 16-row tiles and keeps everything of a tile in
// registers.  Lane l (i = l % 16, g = l / 16) loads the 16-byte pieces
// A[row i][16 j + 4 g .. + 3] of its row (j < d / 16).
//  1. Y^T = Z_full^T A_tile^T on 16x16x4 FP32 MFMAs, the contraction index
//     of step (j, e) being column 16 j + 4 g + e: the A operand is
//     Z_full[16 j + 4 g + e][16 nb + i] (LDS), the B operand element e of
//     the lane's piece j.  Accumulator element v of lane l is then
//     Y[row i][16 nb + 4 g + v], which is scaled by 2 w_i.
//  2. G_tile = Y Z_full^T with the contraction index of step (nb, v) taken
//     as 16 nb + 4 g + v: the A operand is exactly accumulator element v of
//     step 1 (Y never leaves the registers), the B operand Z_full[16 db + i]
//     [16 nb + 4 g + v] (LDS).  Element v of the result is G[row 4 g + v]
//     [16 db + i], to which s_r H_full[h(r)][16 db + i] is added before the
//     store.
// Z_full sits in LDS with a row stride of 68 floats (the reads of step 1
// are free of bank conflicts).  NJ = d / 16 rounded up to a multiple of 4:
// pieces past d / 16 load the row's first piece again and are not used.
constexpr int kGradWaves = 8;
constexpr int kZsStride = 68;

template <int KB, int NJ>
__global__ __launch_bounds__(64 * kGradWaves, 4) void bwd_grad_f32_kernel(
    const float* __restrict__ A, int64_t n, int64_t d, int64_t ld, const float* __restrict__ w,
    const float* __restrict__ Zg, const float* __restrict__ Hf, HashParams hp, float* __restrict__ G,
    int64_t ldg) {
  extern __shared__ float zs[];
  const int di = (int)d;
  for (int q = threadIdx.x; q < di * 16 * KB; q += 64 * kGradWaves) {
    const int r = q / (16 * KB), c = q % (16 * KB);
    zs[r * kZsStride + c] = Zg[(int64_t)r * kZCols + c];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, i16 = lane & 15;
  const int nj = di / 16;
  const int64_t ntiles = (n + 15) / 16;
  for (int64_t tile = (int64_t)wave * gridDim.x + blockIdx.x; tile < ntiles;
       tile += (int64_t)gridDim.x * kGradWaves) {
    const int64_t row = tile * 16 + i16;
    const bool ok = row < n;
    const float* rp = A + (ok ? row : 0) * ld + 4 * g;
    float4 a[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) a[j] = *reinterpret_cast<const float4*>(rp + 16 * (j < nj ? j : 0));
    const float ws = ok ? 2.0f * w[row] : 0.0f;
    // the rows this lane stores in step 2: 4 g + v
    int hr[4];
    bool neg[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = tile * 16 + 4 * g + v;
      const uint64_t x = hash_x(hp, (uint64_t)(r < n ? r : 0));
      hr[v] = (int)((uint32_t)x % (uint32_t)hp.r_cs);  // x < P < 2^32
      neg[v] = sign_negative(hp, (uint64_t)(r < n ? r : 0));
    }
    v4f yt[KB];
#pragma unroll
    for (int nb = 0; nb < KB; ++nb) yt[nb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if (j < nj) {
        const float* zr = zs + (16 * j + 4 * g) * kZsStride + i16;
        const float av[4] = {a[j].x, a[j].y, a[j].z, a[j].w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int nb = 0; nb < KB; ++nb)
            yt[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(zr[e * kZsStride + 16 * nb], av[e], yt[nb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int nb = 0; nb < KB; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) yt[nb][v] *= ws;
    // column blocks two at a time (two independent MFMA chains); the H
    // values of the next pair are loaded while a pair is multiplied (an L2
    // round trip per block would otherwise stall the wave 16 times a tile)
    auto load_h = [&](int db, float (&h)[4]) {
      const int cc = 16 * (db < nj ? db : 0) + i16;
#pragma unroll
      for (int v = 0; v < 4; ++v) h[v] = Hf[(int64_t)hr[v] * d + cc];
    };
    float hn0[4], hn1[4];
    load_h(0, hn0);
    load_h(1, hn1);
    for (int db = 0; db < nj; db += 2) {
      float h0[4], h1[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        h0[v] = hn0[v];
        h1[v] = hn1[v];
      }
      load_h(db + 2, hn0);
      load_h(db + 3, hn1);
      const bool two = db + 1 < nj;  // uniform
      const int col0 = 16 * db + i16, col1 = col0 + 16;
      const float* zb0 = zs + col0 * kZsStride + 4 * g;
      const float* zb1 = zs + (two ? col1 : col0) * kZsStride + 4 * g;
      v4f a0 = v4f{0.f, 0.f, 0.f, 0.f}, a1 = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int nb = 0; nb < KB; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(yt[nb][v], zb0[16 * nb + v], a0, 0, 0, 0);
          a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(yt[nb][v], zb1[16 * nb + v], a1, 0, 0, 0);
        }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = tile * 16 + 4 * g + v;
        if (r < n) {
          G[r * ldg + col0] = a0[v] + (neg[v] ? -h0[v] : h0[v]);
          if (two) G[r * ldg + col1] = a1[v] + (neg[v] ? -h1[v] : h1[v]);
        }
      }
    }
  }
}

template <int KB, int NJ>
hipError_t launch_grad_f32(const float* a, int64_t n, int64_t d, int64_t ld, const float* w, const float* z,
                           const float* h, const HashParams& hp, float* out, int64_t ldg, hipStream_t s) {
  auto kern = bwd_grad_f32_kernel<KB, NJ>;
  const size_t lds = (size_t)d * kZsStride * sizeof(float);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, num_cu = 0, per_cu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * kGradWaves, lds)) != hipSuccess)
    return e;
  const int64_t ntiles = (n + 15) / 16;
  const int64_t want = (ntiles + kGradWaves - 1) / kGradWaves;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cu * std::max(per_cu, 1)));
  kern<<<(unsigned)blocks, 64 * kGradWaves, lds, s>>>(a, n, d, ld, w, z, h, hp, out, ldg);
  return hipGetLastError();
}

template <int KB>
hipError_t launch_grad_f32_kb(const float* a, int64_t n, int64_t d, int64_t ld, const float* w, const float* z,
                              const float* h, const HashParams& hp, float* out, int64_t ldg, hipStream_t s) {
  switch ((d / 16 + 3) / 4) {
    case 1: return launch_grad_f32<KB, 4>(a, n, d, ld, w, z, h, hp, out, ldg, s);
    case 2: return launch_grad_f32<KB, 8>(a, n, d, ld, w, z, h, hp, out, ldg, s);
    case 3: return launch_grad_f32<KB, 12>(a, n, d, ld, w, z, h, hp, out, ldg, s);
    default: return launch_grad_f32<KB, 16>(a, n, d, ld, w, z, h, hp, out, ldg, s);
  }
}

// C = A^T (w o Y) for FP32 A under the same conditions.  Wave w of a
// workgroup of KB * S waves owns column block nb = w % KB of C (d x 16, in
// its registers for the whole pass) and tile stream w / KB; S is chosen so
// that the waves spread evenly over the four SIMDs.  Per 16-row tile:
//  1. column block nb of Y^T as in bwd_grad_f32_kernel (Z_full's block nb
//     only), scaled by w_i;
//  2. through a per-wave LDS block, so that lane l holds Yw[row 4 s + g]
//     [16 nb + i] (s < 4);
//  3. C^T[block nb] += Yw^T A_tile on 16x16x4 FP32 MFMAs contracting over
//     the tile's rows (step s takes row 4 s + g).  The B operand needs A
//     with the row in the lane group, so the tile is read a second time in
//     that layout, 16 bytes per lane: lane l loads A[row 4 s + g][64 q +
//     4 i .. + 3], and column block (q, e) of C^T is the set of columns
//     64 q + 4 jj + e (jj < 16), un-permuted when C is written out.
// The KB waves of a stream read the same tile at about the same time, so A
// comes from HBM once and from L2 otherwise; the second reads are issued
// after step 1, when the pieces are dead (fewer registers, more waves).  At
// the end the streams add their C into LDS in stream order and the
// workgroup writes one partial (the layout and reduction of
// bwd_gram_kernel).
constexpr int kYtStride = 80;  // floats per row of the per-wave Y block (16 mod 64 words)

// Tile streams per workgroup: waves spread evenly over the four SIMDs within
// the registers C needs; at d <= 64 (NJ = 4) the waves are small and 16 fit.
template <int KB, int NJ>
constexpr int gram_streams() { return NJ <= 4 ? 16 / KB : (KB == 3 ? 4 : (KB == 1 ? 4 : 2)); }

template <int KB, int NJ>
__global__ __launch_bounds__((64 * KB * gram_streams<KB, NJ>()), (KB * gram_streams<KB, NJ>() / 4)) void bwd_gram_f32_kernel(
    const float* __restrict__ A, int64_t n, int64_t d, int64_t ld, const float* __restrict__ w,
    const float* __restrict__ Zg, float* __restrict__ partials) {
  constexpr int S = gram_streams<KB, NJ>();
  constexpr int NQ = NJ / 4;  // 64-column groups
  constexpr int kT = 64 * KB * S;
  extern __shared__ float smem_f[];
  float* zs = smem_f;                            // d x kZsStride (then C)
  float* ybuf = smem_f + (size_t)d * kZsStride;  // KB S x 16 x kYtStride
  const int di = (int)d;
  for (int q = threadIdx.x; q < di * 16 * KB; q += kT) {
    const int r = q / (16 * KB), c = q % (16 * KB);
    zs[r * kZsStride + c] = Zg[(int64_t)r * kZCols + c];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nb = wave % KB, stream = wave / KB;
  const int g = lane >> 4, i16 = lane & 15;
  const int nj = di / 16;
  float* yb = ybuf + wave * 16 * kYtStride;
  v4f cacc[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) cacc[q][e] = v4f{0.f, 0.f, 0.f, 0.f};

  const int64_t ntiles = (n + 15) / 16;
  // The KB waves of a stream read the same tile; a barrier per round keeps
  // them (and the streams) within one tile of each other, so the tile is
  // fetched from HBM once and found in L2 by the others (drifting apart,
  // each wave fetched its own copy: 2.8x the bytes of A).  The trip count
  // is the workgroup's, the same for every wave.
  for (int64_t t0 = blockIdx.x; t0 < ntiles; t0 += (int64_t)gridDim.x * S) {
    const int64_t tile = t0 + (int64_t)stream * gridDim.x;
    if (tile < ntiles) {
    // the tile's pieces, row i16 in the lanes: 16 j + 4 g .. + 3
    const int64_t row = tile * 16 + i16;
    const float* rp = A + (row < n ? row : 0) * ld + 4 * g;
    float4 a[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) a[j] = *reinterpret_cast<const float4*>(rp + 16 * (j < nj ? j : 0));
    const float ws = row < n ? (w != nullptr ? w[row] : 1.0f) : 0.0f;  // w = null: all ones
    v4f yt = v4f{0.f, 0.f, 0.f, 0.f};
    const float* zc = zs + 4 * g * kZsStride + 16 * nb + i16;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if (j < nj) {
        const float av[4] = {a[j].x, a[j].y, a[j].z, a[j].w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
          yt = __builtin_amdgcn_mfma_f32_16x16x4f32(zc[(16 * j + e) * kZsStride], av[e], yt, 0, 0, 0);
      }
    }
    // the tile again, rows in the lane group (columns 64 q + 4 i16 .. + 3;
    // pieces past d read column 0 and are dropped)
    float4 rl[4][NQ];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int64_t r = tile * 16 + 4 * s4 + g;
      const float* rq = A + (r < n ? r : 0) * ld;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int c = 64 * q + 4 * i16;
        rl[s4][q] = *reinterpret_cast<const float4*>(rq + (c < di ? c : 0));
      }
    }
    // Yw[row i16][16 nb + 4 g + v] -> LDS, back as Yw[row 4 s + g][16 nb + i16]
    // (the wave's own block: LDS serves a wave's accesses in order)
    *reinterpret_cast<float4*>(yb + i16 * kYtStride + 4 * g) =
        make_float4(yt[0] * ws, yt[1] * ws, yt[2] * ws, yt[3] * ws);
    float yop[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) yop[s4] = yb[(4 * s4 + g) * kYtStride + i16];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (q * 4 < nj) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const float rv[4] = {rl[s4][q].x, rl[s4][q].y, rl[s4][q].z, rl[s4][q].w};
#pragma unroll
          for (int e = 0; e < 4; ++e)
            cacc[q][e] = __builtin_amdgcn_mfma_f32_16x16x4f32(yop[s4], rv[e], cacc[q][e], 0, 0, 0);
        }
      }
    }
    }
    __builtin_amdgcn_s_barrier();
  }
  // C[64 q + 4 i16 + e][16 nb + 4 g + v] = cacc[q][e][v]; streams add in order
  __syncthreads();  // every wave is done with zs
  float* red = zs;  // d x 64
  for (int st = 0; st < S; ++st) {
    if (stream == st) {
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = 64 * q + 4 * i16 + e;
          if (c < di) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              float* dst = red + c * kZCols + 16 * nb + 4 * g + v;
              *dst = st == 0 ? cacc[q][e][v] : *dst + cacc[q][e][v];
            }
          }
        }
    }
    __syncthreads();
  }
  float* out = partials + (int64_t)blockIdx.x * d * kZCols;
  for (int q = threadIdx.x; q < di * 16 * KB; q += kT) {
    const int r = q / (16 * KB), c = q % (16 * KB);
    out[(int64_t)r * kZCols + c] = red[r * kZCols + c];
  }
}

template <int KB, int NJ>
hipError_t launch_gram_f32(const float* a, int64_t n, int64_t d, int64_t ld, const float* w, const float* z,
                           float* partials, int groups, hipStream_t s) {
  auto kern = bwd_gram_f32_kernel<KB, NJ>;
  constexpr int kWavesWg = KB * gram_streams<KB, NJ>();
  const size_t lds = ((size_t)d * kZsStride + (size_t)kWavesWg * 16 * kYtStride) * sizeof(float);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  kern<<<(unsigned)groups, 64 * kWavesWg, lds, s>>>(a, n, d, ld, w, z, partials);
  return hipGetLastError();
}

template <int KB>
hipError_t launch_gram_f32_kb(const float* a, int64_t n, int64_t d, int64_t ld, const float* w, const float* z,
                              float* partials, int groups, hipStream_t s) {
  switch ((d / 16 + 3) / 4) {
    case 1: return launch_gram_f32<KB, 4>(a, n, d, ld, w, z, partials, groups, s);
    case 2: return launch_gram_f32<KB, 8>(a, n, d, ld, w, z, partials, groups, s);
    case 3: return launch_gram_f32<KB, 12>(a, n, d, ld, w, z, partials, groups, s);
    default: return launch_gram_f32<KB, 16>(a, n, d, ld, w, z, partials, groups, s);
  }
}

// Workgroups of the C pass: one per compute unit of an MI355X (each holds
// ~130 KB of LDS, so one fits per CU).  A constant, so that the partial-sum
// order, hence the bits of C, do not depend on the device queried.
constexpr int kGramGroups = 256;

template <typename T, typename K>
hipError_t launch_with_lds(K kern, dim3 grid, size_t lds, hipStream_t s) {
  (void)grid;
  (void)s;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

template <typename T>
hipError_t gram_typed(const void* A, int64_t n, int64_t d, int64_t ld, int64_t k, const void* w, const void* Zfull,
                      void* partials, int groups, double* C64, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (d % 16 == 0 && d <= 256 && k <= 64) {
      const float* a = static_cast<const float*>(A);
      const float* wv = static_cast<const float*>(w);
      const float* z = static_cast<const float*>(Zfull);
      float* p = static_cast<float*>(partials);
      hipError_t e;
      switch ((k + 15) / 16) {
        case 1: e = launch_gram_f32_kb<1>(a, n, d, ld, wv, z, p, groups, s); break;
        case 2: e = launch_gram_f32_kb<2>(a, n, d, ld, wv, z, p, groups, s); break;
        case 3: e = launch_gram_f32_kb<3>(a, n, d, ld, wv, z, p, groups, s); break;
        default: e = launch_gram_f32_kb<4>(a, n, d, ld, wv, z, p, groups, s); break;
      }
      if (e != hipSuccess) return e;
      const int64_t total = d * k;
      bwd_reduce_kernel<T><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(static_cast<const T*>(partials), groups,
                                                                            d, k, C64);
      return hipGetLastError();
    }
  }
  const TileGeom g = tile_geom<T>(d, k);
  const bool zlds = lds_bytes<T>(g, true) <= 144 * 1024;
  const size_t lds = lds_bytes<T>(g, zlds);
  const int total_blocks = (g.d16 / 16) * g.kb;
  const int per_slice = kWaves * kMaxCBlocks;
  const int slices = (total_blocks + per_slice - 1) / per_slice;
  const dim3 grid((unsigned)groups, (unsigned)slices);
  const T* a = static_cast<const T*>(A);
  const T* wv = static_cast<const T*>(w);
  const T* z = static_cast<const T*>(Zfull);
  T* p = static_cast<T*>(partials);
  hipError_t e;
  if (zlds) {
    auto kern = bwd_gram_kernel<T, true>;
    if ((e = launch_with_lds<T>(kern, grid, lds, s)) != hipSuccess) return e;
    kern<<<grid, kThreads, lds, s>>>(a, n, d, ld, wv, z, g, per_slice, p);
  } else {
    auto kern = bwd_gram_kernel<T, false>;
    if ((e = launch_with_lds<T>(kern, grid, lds, s)) != hipSuccess) return e;
    kern<<<grid, kThreads, lds, s>>>(a, n, d, ld, wv, z, g, per_slice, p);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t total = d * k;
  bwd_reduce_kernel<T><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(p, groups, d, k, C64);
  return hipGetLastError();
}

template <typename T>
hipError_t grad_typed(const void* A, int64_t n, int64_t d, int64_t ld, int64_t k, const void* w, const void* Zfull,
                      const void* Hfull, const HashParams& hp, void* G, int64_t ldg, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    // rows are 16-byte aligned (the interface requires it), so the pieces are
    if (d % 16 == 0 && d <= 256 && k <= 64) {
      const float* a = static_cast<const float*>(A);
      const float* wv = static_cast<const float*>(w);
      const float* z = static_cast<const float*>(Zfull);
      const float* h = static_cast<const float*>(Hfull);
      float* out = static_cast<float*>(G);
      switch ((k + 15) / 16) {
        case 1: return launch_grad_f32_kb<1>(a, n, d, ld, wv, z, h, hp, out, ldg, s);
        case 2: return launch_grad_f32_kb<2>(a, n, d, ld, wv, z, h, hp, out, ldg, s);
        case 3: return launch_grad_f32_kb<3>(a, n, d, ld, wv, z, h, hp, out, ldg, s);
        default: return launch_grad_f32_kb<4>(a, n, d, ld, wv, z, h, hp, out, ldg, s);
      }
    }
  }
  const TileGeom g = tile_geom<T>(d, k);
  const bool zlds = lds_bytes<T>(g, true) <= 144 * 1024;
  const size_t lds = lds_bytes<T>(g, zlds);
  const int64_t ntiles = (n + g.TM - 1) / g.TM;
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(ntiles, 4096)));
  const T* a = static_cast<const T*>(A);
  const T* wv = static_cast<const T*>(w);
  const T* z = static_cast<const T*>(Zfull);
  const T* h = static_cast<const T*>(Hfull);
  T* out = static_cast<T*>(G);
  hipError_t e;
  if (zlds) {
    auto kern = bwd_grad_kernel<T, true>;
    if ((e = launch_with_lds<T>(kern, grid, lds, s)) != hipSuccess) return e;
    kern<<<grid, kThreads, lds, s>>>(a, n, d, ld, wv, z, h, hp, g, out, ldg);
  } else {
    auto kern = bwd_grad_kernel<T, false>;
    if ((e = launch_with_lds<T>(kern, grid, lds, s)) != hipSuccess) return e;
    kern<<<grid, kThreads, lds, s>>>(a, n, d, ld, wv, z, h, hp, g, out, ldg);
  }
  return hipGetLastError();
}

// ---- LS-HRN-exact (Algorithm 7) helpers -----------------------------------------
// B_K[i][j] = C[perm[i]][perm[j]] for i, j < r, else 0 (d x d).
__global__ void gather_bk_kernel(int64_t d, const int32_t* __restrict__ perm, const int64_t* __restrict__ rank,
                                 const double* __restrict__ C, double* __restrict__ B) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  const int64_t i = idx / d, j = idx % d, r = *rank;
  B[idx] = (i < r && j < r) ? C[(int64_t)perm[i] * d + perm[j]] : 0.0;
}

// permc[j] = perm[perm2[j]]: column ids of A in the order of the Cholesky of B_K.
__global__ void compose_perm_kernel(int64_t d, const int32_t* __restrict__ perm, const int32_t* __restrict__ perm2,
                                    int32_t* __restrict__ permc) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < d) permc[j] = perm[perm2[j]];
}

// ---- small FP64 helpers of the core --------------------------------------------
// Zbar[j][c] = j < r ? 2 C64[perm[j]][c] : 0.
__global__ void gather_zbar_kernel(int64_t d, int64_t k, const int32_t* __restrict__ perm,
                                   const int64_t* __restrict__ rank, const double* __restrict__ C64,
                                   double* __restrict__ Zbar) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * k) return;
  const int64_t j = idx / k, c = idx % k;
  Zbar[idx] = j < *rank ? 2.0 * C64[(int64_t)perm[j] * k + c] : 0.0;
}

// X <- -triu(X) (d x d)
__global__ void neg_triu_kernel(int64_t d, double* __restrict__ X) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  const int64_t i = idx / d, j = idx % d;
  X[idx] = j >= i ? -X[idx] : 0.0;
}

// out = tril(M) + tril(M, -1)^T
__global__ void copyltu_kernel(int64_t d, const double* __restrict__ M, double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  const int64_t i = idx / d, j = idx % d;
  out[idx] = i >= j ? M[i * d + j] : M[j * d + i];
}

__global__ void identity_kernel(int64_t d, double* __restrict__ I) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  I[idx] = (idx / d == idx % d) ? 1.0 : 0.0;
}

// AtK[i][j] = j < r ? At[i][perm[j]] : 0   (m x d)
__global__ void gather_cols_kernel(int64_t m, int64_t d, const int32_t* __restrict__ perm,
                                   const int64_t* __restrict__ rank, const double* __restrict__ At,
                                   double* __restrict__ AtK) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * d) return;
  const int64_t i = idx / d, j = idx % d;
  AtK[idx] = j < *rank ? At[i * d + perm[j]] : 0.0;
}

// Hf[b][perm[j]] = j < r ? H[b][j] : 0   (r_cs x d), in the gradient's type
template <typename T>
__global__ void scatter_h_kernel(int64_t rows, int64_t d, const int32_t* __restrict__ perm,
                                 const int64_t* __restrict__ rank, const double* __restrict__ H, T* __restrict__ Hf) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * d) return;
  const int64_t b = idx / d, j = idx % d;
  Hf[b * d + perm[j]] = (T)(j < *rank ? H[idx] : 0.0);
}

unsigned blocks_for(int64_t total) { return (unsigned)((total + 255) / 256); }

}  // namespace

int bwd_groups(int dtype, int64_t n, int64_t d, int64_t k) {
  const int64_t tm = dtype == 0 ? tile_geom<double>(d, k).TM : tile_geom<float>(d, k).TM;
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + tm - 1) / tm, kGramGroups));
}

hipError_t launch_bwd_gram(int dtype, const void* A, int64_t n, int64_t d, int64_t ld, int64_t k, const void* w,
                           const void* Zfull, void* partials, int groups, double* C64, hipStream_t s) {
  if (dtype == 0) return gram_typed<double>(A, n, d, ld, k, w, Zfull, partials, groups, C64, s);
  if (dtype == 1) return gram_typed<float>(A, n, d, ld, k, w, Zfull, partials, groups, C64, s);
  return hipErrorInvalidValue;
}

hipError_t launch_bwd_grad(int dtype, const void* A, int64_t n, int64_t d, int64_t ld, int64_t k, const void* w,
                           const void* Zfull, const void* Hfull, const HashParams& hp, void* G, int64_t ldg,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (dtype == 0) return grad_typed<double>(A, n, d, ld, k, w, Zfull, Hfull, hp, G, ldg, s);
  if (dtype == 1) return grad_typed<float>(A, n, d, ld, k, w, Zfull, Hfull, hp, G, ldg, s);
  return hipErrorInvalidValue;
}

hipError_t launch_gather_bk(int64_t d, const int32_t* perm, const int64_t* rank, const double* C, double* B,
                            hipStream_t s) {
  gather_bk_kernel<<<(unsigned)((d * d + 255) / 256), 256, 0, s>>>(d, perm, rank, C, B);
  return hipGetLastError();
}

hipError_t launch_compose_perm(int64_t d, const int32_t* perm, const int32_t* perm2, int32_t* permc, hipStream_t s) {
  compose_perm_kernel<<<(unsigned)((d + 255) / 256), 256, 0, s>>>(d, perm, perm2, permc);
  return hipGetLastError();
}

hipError_t launch_gather_zbar(int64_t d, int64_t k, const int32_t* perm, const int64_t* rank, const double* C64,
                              double* Zbar, hipStream_t s) {
  gather_zbar_kernel<<<blocks_for(d * k), 256, 0, s>>>(d, k, perm, rank, C64, Zbar);
  return hipGetLastError();
}
hipError_t launch_neg_triu(int64_t d, double* X, hipStream_t s) {
  neg_triu_kernel<<<blocks_for(d * d), 256, 0, s>>>(d, X);
  return hipGetLastError();
}
hipError_t launch_copyltu(int64_t d, const double* M, double* out, hipStream_t s) {
  copyltu_kernel<<<blocks_for(d * d), 256, 0, s>>>(d, M, out);
  return hipGetLastError();
}
hipError_t launch_identity(int64_t d, double* I, hipStream_t s) {
  identity_kernel<<<blocks_for(d * d), 256, 0, s>>>(d, I);
  return hipGetLastError();
}
hipError_t launch_gather_cols(int64_t m, int64_t d, const int32_t* perm, const int64_t* rank, const double* At,
                              double* AtK, hipStream_t s) {
  gather_cols_kernel<<<blocks_for(m * d), 256, 0, s>>>(m, d, perm, rank, At, AtK);
  return hipGetLastError();
}
hipError_t launch_scatter_h(int dtype, int64_t rows, int64_t d, const int32_t* perm, const int64_t* rank,
                            const double* H, void* Hf, hipStream_t s) {
  if (dtype == 0)
    scatter_h_kernel<double><<<blocks_for(rows * d), 256, 0, s>>>(rows, d, perm, rank, H, static_cast<double*>(Hf));
  else
    scatter_h_kernel<float><<<blocks_for(rows * d), 256, 0, s>>>(rows, d, perm, rank, H, static_cast<float*>(Hf));
  return hipGetLastError();
}

size_t bwd_elem_size(int dtype) { return dtype == 0 ? sizeof(double) : sizeof(float); }

}  // namespace lev

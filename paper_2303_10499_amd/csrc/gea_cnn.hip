// gea_cnn.hip -- bfloat16 matrix-core kernels of the learned initial guess /
// preconditioner network (forward, backward, Adam) and its C ABI
// (include/gea_learned.h).
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (gfx950):
//   forward / backward-data:  M = cells, N = output channels,
//                             K = taps x input channels (zero-padded to 32);
//   backward-weight:          M = output channels, N = taps x input channels,
//                             K = cells, split over workgroups, the splits
//                             summed in a fixed order by a second kernel.
// Operand lane layout of the 16x16x32 instruction (checked on the device):
// lane l holds A[m = l%16][k = 8*(l/16) + i] and B[k = 8*(l/16) + i][n = l%16]
// for i = 0..7, and D[m = 4*(l/16) + i][n = l%16] for i = 0..3.  With
// channels-last activations and input channels padded to a multiple of 8,
// each lane's 8 K-values of one tap are 16 contiguous bytes.
// Backward-data is the forward kernel run on the output gradient with the
// weights flipped in space and transposed in channels.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>

#include "../../include/gea_learned.h"
#include "gea_cnn_internal.h"
#include "gea_reduce.h"

namespace gea {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMT = 2;  // 16-cell M tiles per wave in the convolution
constexpr int kPixPerSplit = 512;

__device__ __forceinline__ bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite values)
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 load8(const bf16_t* p) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, u);
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

template <int NDIM>
struct Taps {
  static constexpr int n = NDIM == 2 ? 9 : 27;
};

// neighbour of cell (i, j, k) at tap t, or -1 outside the grid
template <int NDIM>
__device__ __forceinline__ int neighbor(const CnnDims& d, int i, int j, int k, int t) {
  int dx, dy, dz;
  if (NDIM == 2) {
    dz = t / 3 - 1;
    dx = t % 3 - 1;
    dy = 0;
  } else {
    dz = t / 9 - 1;
    dy = (t / 3) % 3 - 1;
    dx = t % 3 - 1;
  }
  const int a = i + dx, b = j + dy, c = k + dz;
  if (a < 0 || a >= d.nx || b < 0 || b >= d.ny || c < 0 || c >= d.nz) return -1;
  return a + d.nx * (b + d.ny * c);
}

template <int NDIM>
__device__ __forceinline__ void coords(const CnnDims& d, int p, int& i, int& j, int& k) {
  i = p % d.nx;
  const int r = p / d.nx;
  if (NDIM == 2) {
    j = 0;
    k = r;
  } else {
    j = r % d.ny;
    k = r / d.ny;
  }
}

// MODE 0: +bias, ReLU, bf16 out; 1: +bias, FP32 out (first ycount channels);
// 2: no bias, FP32 out (backward-data).
template <int NDIM, int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(CnnDims d, const bf16_t* __restrict__ X,
                                              const bf16_t* __restrict__ W,
                                              const float* __restrict__ bias, void* __restrict__ Y,
                                              int ystride, int ycount) {
  constexpr int NT = Taps<NDIM>::n;
  constexpr int KC = (NT * CIN + 31) / 32;
  constexpr int KPAD = KC * 32;
  constexpr int NTILE = COUT / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int pbase = (blockIdx.x * 4 + wave) * (16 * kMT);
  int pi[kMT], pj[kMT], pk[kMT];
  bool pv[kMT];
#pragma unroll
  for (int mt = 0; mt < kMT; ++mt) {
    const int p = pbase + mt * 16 + r;
    pv[mt] = p < d.npix;
    coords<NDIM>(d, pv[mt] ? p : 0, pi[mt], pj[mt], pk[mt]);
  }
  f32x4 acc[kMT][NTILE];
#pragma unroll
  for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int kc = 0; kc < KC; ++kc) {
    const int k = kc * 32 + 8 * g;
    const int t = k / CIN, ci = k % CIN;
    bf16x8 bw[NTILE];
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt)
      bw[nt] = (t < NT) ? load8(W + (size_t)(nt * 16 + r) * KPAD + k) : zero8();
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt) {
      bf16x8 a = zero8();
      if (t < NT && pv[mt]) {
        const int q = neighbor<NDIM>(d, pi[mt], pj[mt], pk[mt], t);
        if (q >= 0) a = load8(X + (size_t)q * CIN + ci);
      }
#pragma unroll
      for (int nt = 0; nt < NTILE; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[nt], acc[mt][nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = pbase + mt * 16 + 4 * g + i;
        const int co = nt * 16 + r;
        if (p < d.npix && co < ycount) {
          float v = acc[mt][nt][i];
          if (MODE < 2) v += bias[co];
          if (MODE == 0) {
            v = fmaxf(v, 0.f);
            reinterpret_cast<bf16_t*>(Y)[(size_t)p * ystride + co] = f2bf(v);
          } else {
            reinterpret_cast<float*>(Y)[(size_t)p * ystride + co] = v;
          }
        }
      }
}

// Output tile of the forward convolution: TX x TY x TZ cells, staged with a
// one-cell halo in LDS.  A 16-cell M tile is 16 consecutive x cells; wave w
// owns the M tiles of z-row w (3D: the TY rows of that z plane; 2D: the
// TX/16 segments of that row), so every weight chunk a wave loads serves
// MTW M tiles.  For a concatenated input [up(A), X] the fine part X is
// staged per fine cell and the coarse part A once per coarse cell (CHX x
// CHY x CHZ coarse cells cover the fine tile and its halo).
template <int NDIM, int CIN, int CA>
struct ConvTile {
  static constexpr int TX = NDIM == 3 ? 16 : 64;
  static constexpr int TY = NDIM == 3 ? 4 : 1;
  static constexpr int TZ = (NDIM == 3 && CIN > 64) ? 2 : 4;
  static constexpr int HX = TX + 2, HY = NDIM == 3 ? TY + 2 : 1, HZ = TZ + 2;
  static constexpr int HP = HX * HY * HZ;              // staged fine cells
  static constexpr int CF = CIN - CA;                  // channels staged per fine cell
  static constexpr int FSP = CF + 8;                   // LDS stride per fine cell (bf16), padded against bank conflicts
  static constexpr int CHX = TX / 2 + 2, CHY = NDIM == 3 ? TY / 2 + 2 : 1, CHZ = TZ / 2 + 2;
  static constexpr int CHP = CA > 0 ? CHX * CHY * CHZ : 0;  // staged coarse cells
  static constexpr int CSP = CA + 8;                   // LDS stride per coarse cell
  static constexpr int LDS = HP * FSP + CHP * CSP;     // bf16 elements
  static constexpr int MT = (TX / 16) * TY * TZ;       // M tiles per workgroup
  static constexpr int MTW = MT / 4;                   // per wave
};

// bf16 output of a convolution tile through LDS: every lane writes its
// accumulator values (+bias, ReLU) as [cell][channel] into `buf` (PX cells of
// the tile, COUT channels), then the workgroup stores whole 16-byte channel
// groups, consecutive lanes covering consecutive bytes of Y.  The caller
// synchronises before (buf may alias the staged input).
template <int NDIM, int COUT, int MTW, int TX, int TY, int TZ>
__device__ __forceinline__ void store_relu_tile(const f32x4 (&acc)[MTW][COUT / 16], const float* __restrict__ bias,
                                                bf16_t* buf, const CnnDims& d, int ox, int oy, int oz,
                                                bf16_t* __restrict__ Y) {
  constexpr int PX = TX * TY * TZ;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
#pragma unroll
  for (int m = 0; m < MTW; ++m) {
    const int mt = wave * MTW + m;
#pragma unroll
    for (int nt = 0; nt < COUT / 16; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = mt * 16 + 4 * g + i;  // cell of the tile: M tile mt, row position 4g+i
        const int co = nt * 16 + r;
        buf[q * COUT + co] = f2bf(fmaxf(acc[m][nt][i] + bias[co], 0.f));
      }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < PX * (COUT / 8); e += 256) {
    const int q = e / (COUT / 8), c8 = (e % (COUT / 8)) * 8;
    const int mt = q / 16, x16 = q % 16;
    const int seg = mt % (TX / 16), row = mt / (TX / 16);
    const int gx = ox + seg * 16 + x16;
    const int gy = oy + (NDIM == 3 ? row % TY : 0), gz = oz + (NDIM == 3 ? row / TY : row);
    if (gx < d.nx && gy < d.ny && gz < d.nz) {
      const size_t p = (size_t)gx + (size_t)d.nx * (gy + (size_t)d.ny * gz);
      *reinterpret_cast<uint4*>(Y + p * COUT + c8) = *reinterpret_cast<const uint4*>(buf + q * COUT + c8);
    }
  }
}

// Forward convolution through an LDS-staged input tile.  CA = 0: input X
// with CIN channels; CA > 0: the channel concatenation [up(A), X] of a
// coarse tensor A (CA channels, nearest-upsampled) and a fine tensor X
// (CIN - CA channels).  Output: +bias, ReLU, bf16.
template <int NDIM, int CIN, int COUT, int CA>
__global__ __launch_bounds__(256) void k_conv_t(CnnDims d, const bf16_t* __restrict__ X,
                                                const bf16_t* __restrict__ A,
                                                const bf16_t* __restrict__ W,
                                                const float* __restrict__ bias,
                                                bf16_t* __restrict__ Y) {
  using T = ConvTile<NDIM, CIN, CA>;
  constexpr int NT = Taps<NDIM>::n;
  constexpr int KC = (NT * CIN + 31) / 32;
  constexpr int KPAD = KC * 32;
  constexpr int NTILE = COUT / 16;
  constexpr int CF = T::CF;
  constexpr int PX = T::TX * T::TY * T::TZ;
  constexpr int LDSN = T::LDS > PX * COUT ? T::LDS : PX * COUT;  // input tile, then output tile
  __shared__ __attribute__((aligned(16))) bf16_t sIn[LDSN];
  const int ntx = (d.nx + T::TX - 1) / T::TX;
  const int nty = NDIM == 3 ? (d.ny + T::TY - 1) / T::TY : 1;
  // XCD-aware order: neighbouring tiles (which re-read each other's halo
  // cells) run on the same XCD and share its L2
  const int b = xcd_block();
  const int ox = (b % ntx) * T::TX;
  const int oy = NDIM == 3 ? ((b / ntx) % nty) * T::TY : 0;
  const int oz = (b / (ntx * nty)) * T::TZ;
  // ---- stage the tile and its halo (zeros outside the grid); batches of
  // kStage 16-byte loads are issued before their LDS writes
  constexpr int NEF = T::HP * (CF / 8);
  constexpr int NE = NEF + T::CHP * (CA / 8);
  constexpr int kStage = 8;
  const int nxc = d.nx / 2, nyc = NDIM == 3 ? d.ny / 2 : 1, nzc = d.nz / 2;
  // (LDS offset, source) of staging element e; src == nullptr: zero
  auto locate = [&](int e, int& lds) -> const bf16_t* {
    if (e < NEF) {
      const int hp = e / (CF / 8), c8 = (e % (CF / 8)) * 8;
      lds = hp * T::FSP + c8;
      const int hx = hp % T::HX, hy = (hp / T::HX) % T::HY, hz = hp / (T::HX * T::HY);
      const int gx = ox + hx - 1, gy = NDIM == 3 ? oy + hy - 1 : 0, gz = oz + hz - 1;
      if (gx < 0 || gx >= d.nx || gy < 0 || gy >= d.ny || gz < 0 || gz >= d.nz) return nullptr;
      return X + (size_t)(gx + d.nx * (gy + d.ny * gz)) * CF + c8;
    }
    const int e2 = e - NEF;
    const int cp = e2 / (CA > 0 ? CA / 8 : 1), c8 = (e2 % (CA > 0 ? CA / 8 : 1)) * 8;
    lds = T::HP * T::FSP + cp * T::CSP + c8;
    const int cx = cp % T::CHX, cy = (cp / T::CHX) % T::CHY, cz = cp / (T::CHX * T::CHY);
    const int gx = ox / 2 - 1 + cx, gy = NDIM == 3 ? oy / 2 - 1 + cy : 0, gz = oz / 2 - 1 + cz;
    if (gx < 0 || gx >= nxc || gy < 0 || gy >= nyc || gz < 0 || gz >= nzc) return nullptr;
    return A + (size_t)(gx + nxc * (gy + nyc * gz)) * (CA > 0 ? CA : 1) + c8;
  };
  for (int e0 = threadIdx.x; e0 < NE; e0 += 256 * kStage) {
    uint4 v[kStage];
    int lds[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      v[u] = make_uint4(0, 0, 0, 0);
      lds[u] = -1;
      const int e = e0 + 256 * u;
      if (e < NE) {
        // groups of 8 bf16 channels start on 16-byte boundaries (channel counts are multiples of 8)
        const bf16_t* src = locate(e, lds[u]);
        if (src) v[u] = *reinterpret_cast<const uint4*>(__builtin_assume_aligned(src, 16));
      }
    }
#pragma unroll
    for (int u = 0; u < kStage; ++u)
      if (lds[u] >= 0) *reinterpret_cast<uint4*>(sIn + lds[u]) = v[u];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  // local coordinates (lane r) and staged fine cell of each of the wave's M tiles
  int lxm[T::MTW], lym[T::MTW], lzm[T::MTW], pix[T::MTW];
#pragma unroll
  for (int m = 0; m < T::MTW; ++m) {
    const int mt = wave * T::MTW + m;
    const int seg = mt % (T::TX / 16), row = mt / (T::TX / 16);
    lxm[m] = seg * 16 + r;
    lym[m] = NDIM == 3 ? row % T::TY : 0;
    lzm[m] = NDIM == 3 ? row / T::TY : row;
    pix[m] = (lxm[m] + 1) + T::HX * ((NDIM == 3 ? lym[m] + 1 : 0) + T::HY * (lzm[m] + 1));
  }
  f32x4 acc[T::MTW][NTILE];
#pragma unroll
  for (int m = 0; m < T::MTW; ++m)
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt) acc[m][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  // operands of one 32-wide K chunk: weights (global, cached) and the
  // wave's M tiles (LDS); the next chunk's operands are loaded before the
  // current chunk's MFMAs are issued
  auto load_chunk = [&](int kc, bf16x8(&a)[T::MTW], bf16x8(&bw)[NTILE]) {
    const int k = kc * 32 + 8 * g;
    const int t = k / CIN, ci = k % CIN;
    const bool tap = t < NT;
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt)
      bw[nt] = tap ? load8(W + (size_t)(nt * 16 + r) * KPAD + k) : zero8();
    const int dx = t % 3 - 1;
    const int dy = NDIM == 3 ? (t / 3) % 3 - 1 : 0;
    const int dz = NDIM == 3 ? t / 9 - 1 : t / 3 - 1;
    const bool coarse = ci < CA;
    const int offf = (dx + T::HX * (dy + T::HY * dz)) * T::FSP + (ci - CA);
#pragma unroll
    for (int m = 0; m < T::MTW; ++m) {
      int addr = pix[m] * T::FSP + offf;
      if (CA > 0) {
        const int cx = (lxm[m] + dx + 2) >> 1;
        const int cy = NDIM == 3 ? (lym[m] + dy + 2) >> 1 : 0;
        const int cz = (lzm[m] + dz + 2) >> 1;
        const int ca = T::HP * T::FSP + (cx + T::CHX * (cy + T::CHY * cz)) * T::CSP + ci;
        addr = coarse ? ca : addr;
      }
      a[m] = tap ? __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(sIn + addr)) : zero8();
    }
  };
  bf16x8 a0[T::MTW], b0[NTILE], a1[T::MTW], b1[NTILE];
  load_chunk(0, a0, b0);
#pragma unroll
  for (int kc = 0; kc < KC; kc += 2) {
    if (kc + 1 < KC) load_chunk(kc + 1, a1, b1);
#pragma unroll
    for (int m = 0; m < T::MTW; ++m)
#pragma unroll
      for (int nt = 0; nt < NTILE; ++nt)
        acc[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[m], b0[nt], acc[m][nt], 0, 0, 0);
    if (kc + 1 < KC) {
      if (kc + 2 < KC) load_chunk(kc + 2, a0, b0);
#pragma unroll
      for (int m = 0; m < T::MTW; ++m)
#pragma unroll
        for (int nt = 0; nt < NTILE; ++nt)
          acc[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[m], b1[nt], acc[m][nt], 0, 0, 0);
    }
  }
  __syncthreads();  // every wave is done with the staged input
  store_relu_tile<NDIM, COUT, T::MTW, T::TX, T::TY, T::TZ>(acc, bias, sIn, d, ox, oy, oz, Y);
}

// Layer 0: the input has 2 real channels (r/s and c/diag) stored in 8.  Each
// staged cell keeps only those 2 (4 bytes) and K is ordered tap x 2 +
// channel, 54 padded to 64: two 32-wide chunks cover all 27 taps (instead of
// seven chunks of 8-channel taps), each lane's 8 K-values being 4 taps x 2
// channels from four 4-byte LDS reads.  W0 holds the weights in that order.
template <int NDIM>
__global__ __launch_bounds__(256) void k_conv0(CnnDims d, const uint32_t* __restrict__ X2,
                                               const bf16_t* __restrict__ W0,
                                               const float* __restrict__ bias,
                                               bf16_t* __restrict__ Y) {
  using T = ConvTile<NDIM, 8, 0>;
  constexpr int NT = Taps<NDIM>::n;
  constexpr int KC = (NT * 2 + 31) / 32;
  constexpr int KPAD = KC * 32;
  __shared__ uint32_t s2[T::HP];
  __shared__ __attribute__((aligned(16))) bf16_t sOut[T::TX * T::TY * T::TZ * 16];
  const int ntx = (d.nx + T::TX - 1) / T::TX;
  const int nty = NDIM == 3 ? (d.ny + T::TY - 1) / T::TY : 1;
  const int b = xcd_block();
  const int ox = (b % ntx) * T::TX;
  const int oy = NDIM == 3 ? ((b / ntx) % nty) * T::TY : 0;
  const int oz = (b / (ntx * nty)) * T::TZ;
  for (int hp = threadIdx.x; hp < T::HP; hp += 256) {
    const int hx = hp % T::HX, hy = (hp / T::HX) % T::HY, hz = hp / (T::HX * T::HY);
    const int gx = ox + hx - 1, gy = NDIM == 3 ? oy + hy - 1 : 0, gz = oz + hz - 1;
    uint32_t v = 0;
    if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny && gz >= 0 && gz < d.nz)
      v = X2[gx + d.nx * (gy + d.ny * gz)];
    s2[hp] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  int pix[T::MTW];
#pragma unroll
  for (int m = 0; m < T::MTW; ++m) {
    const int mt = wave * T::MTW + m;
    const int seg = mt % (T::TX / 16), row = mt / (T::TX / 16);
    const int lx = seg * 16 + r;
    const int ly = NDIM == 3 ? row % T::TY : 0, lz = NDIM == 3 ? row / T::TY : row;
    pix[m] = (lx + 1) + T::HX * ((NDIM == 3 ? ly + 1 : 0) + T::HY * (lz + 1));
  }
  f32x4 acc[T::MTW];
#pragma unroll
  for (int m = 0; m < T::MTW; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
    const int t0 = kc * 16 + 4 * g;  // first of this lane group's 4 taps
    const bf16x8 bw = load8(W0 + (size_t)r * KPAD + kc * 32 + 8 * g);
    int off[4];
    bool on[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int t = t0 + i;
      on[i] = t < NT;
      const int dx = t % 3 - 1;
      const int dy = NDIM == 3 ? (t / 3) % 3 - 1 : 0;
      const int dz = NDIM == 3 ? t / 9 - 1 : t / 3 - 1;
      off[i] = on[i] ? dx + T::HX * (dy + T::HY * dz) : 0;  // padding taps: a valid cell, value unused
    }
#pragma unroll
    for (int m = 0; m < T::MTW; ++m) {
      uint4 a;
      a.x = on[0] ? s2[pix[m] + off[0]] : 0u;
      a.y = on[1] ? s2[pix[m] + off[1]] : 0u;
      a.z = on[2] ? s2[pix[m] + off[2]] : 0u;
      a.w = on[3] ? s2[pix[m] + off[3]] : 0u;
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), bw, acc[m], 0, 0, 0);
    }
  }
  f32x4 acc1[T::MTW][1];
#pragma unroll
  for (int m = 0; m < T::MTW; ++m) acc1[m][0] = acc[m];
  store_relu_tile<NDIM, 16, T::MTW, T::TX, T::TY, T::TZ>(acc1, bias, sOut, d, ox, oy, oz, Y);
}

// Layer 5 (16 channels -> 1 output) on the vector units, marching along z:
// a workgroup owns a TX x TY column tile (TX cells of a row in 2D) and a
// chunk of KC output planes.  Each input plane, with a one-cell x/y halo, is
// staged once in LDS (two 16-byte halves per cell, the next plane's loads in
// flight while the current one is used); every thread then adds that plane's
// share to the three output planes it touches (taps dz = +1, 0, -1) with
// bf16 pair dot products accumulated in FP32.  An output plane is complete
// and stored once the plane above it has been added.  Work: 16 x taps
// multiply-adds per cell, no padded output channels.
template <int NDIM>
struct Conv5Z {
  static constexpr int TX = NDIM == 3 ? 64 : 256, TY = NDIM == 3 ? 4 : 1, KC = 16;
  static constexpr int HX = TX + 2, HY = NDIM == 3 ? TY + 2 : 1;
  static constexpr int HC = HX * HY;                // staged cells per plane
  static constexpr int NL = (2 * HC + 255) / 256;   // 16-byte loads per thread and plane
};

__device__ __forceinline__ float dot16(const uint4& p, const uint4& q, const uint32_t* __restrict__ w,
                                       float a) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
#define GEA_D2(V, I) a = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, V), \
                                                         __builtin_bit_cast(bf16x2, w[I]), a, false)
  GEA_D2(p.x, 0); GEA_D2(p.y, 1); GEA_D2(p.z, 2); GEA_D2(p.w, 3);
  GEA_D2(q.x, 4); GEA_D2(q.y, 5); GEA_D2(q.z, 6); GEA_D2(q.w, 7);
#undef GEA_D2
  return a;
}

// With scale given, Y receives (float)*scale times the output (the solver's
// scaled correction; the same product as the output scaling kernel).
template <int NDIM>
__global__ __launch_bounds__(256) void k_conv5z(CnnDims d, const bf16_t* __restrict__ X,
                                                const uint32_t* __restrict__ W5,
                                                const float* __restrict__ bias,
                                                float* __restrict__ Y,
                                                const double* __restrict__ scale) {
  using T = Conv5Z<NDIM>;
  __shared__ uint4 sx[2][2][T::HC];  // [slot][channel half][cell]
  const int ntx = (d.nx + T::TX - 1) / T::TX;
  const int nty = NDIM == 3 ? (d.ny + T::TY - 1) / T::TY : 1;
  const int b = xcd_block();
  const int ox = (b % ntx) * T::TX;
  const int oy = NDIM == 3 ? ((b / ntx) % nty) * T::TY : 0;
  const int k0 = (b / (ntx * nty)) * T::KC;
  const int k1 = min(k0 + T::KC, d.nz);
  const int lx = (int)threadIdx.x % T::TX, ly = (int)threadIdx.x / T::TX;
  const int gx = ox + lx, gy = oy + ly;
  const bool act = gx < d.nx && gy < d.ny;
  const size_t plane = (size_t)d.nx * d.ny;
  uint4 v[T::NL];
  // plane k of d0 with its halo; zeros outside the grid.  Every load is made,
  // from an index clamped into the grid, and the zero padding is a select:
  // no branch separates the plane's loads.
  auto fetch = [&](int k) {
    const bool kin = k >= 0 && k < d.nz;
    const size_t kp = (size_t)(k < 0 ? 0 : (k >= d.nz ? d.nz - 1 : k)) * plane;
#pragma unroll
    for (int u = 0; u < T::NL; ++u) {
      const int e = threadIdx.x + 256 * u, h = e & 1;
      const int c = (e >> 1) < T::HC ? (e >> 1) : T::HC - 1;
      const int x = ox + c % T::HX - 1;
      const int y = NDIM == 3 ? oy + c / T::HX - 1 : 0;
      const bool in = kin && (e >> 1) < T::HC && x >= 0 && x < d.nx && y >= 0 && y < d.ny;
      const int xc = x < 0 ? 0 : (x >= d.nx ? d.nx - 1 : x);
      const int yc = y < 0 ? 0 : (y >= d.ny ? d.ny - 1 : y);
      const uint4 t = *reinterpret_cast<const uint4*>(X + (kp + xc + (size_t)d.nx * yc) * 16 + 8 * h);
      v[u] = in ? t : make_uint4(0, 0, 0, 0);
    }
  };
  auto put = [&](int slot) {
#pragma unroll
    for (int u = 0; u < T::NL; ++u) {
      const int e = threadIdx.x + 256 * u, c = e >> 1, h = e & 1;
      if (c < T::HC) sx[slot][h][c] = v[u];
    }
  };
  const float b0 = bias[0];
  const float sc = scale ? (float)*scale : 1.f;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;  // output planes k - 1, k, k + 1 of input plane k
  fetch(k0 - 1);
  put(0);
  lds_barrier();
  int slot = 0;
  for (int k = k0 - 1; k <= k1; ++k) {
    if (k < k1) fetch(k + 1);
    if (k >= 0 && k < d.nz) {
      // the thread's 3 x 3 (2D: 3) neighbours in this plane, one at a time,
      // each into the three tap groups (dz = +1 for output plane k - 1,
      // dz = 0 for k, dz = -1 for k + 1): three independent chains, and
      // only one neighbour's 16 channels live in registers
      constexpr int NC = NDIM == 3 ? 9 : 3;
      constexpr int TZ = NC;  // tap stride of dz
      const bool g0 = k - 1 >= k0, g1 = k >= k0 && k < k1, g2 = k + 1 < k1;
      float e0 = 0.f, e1 = 0.f, e2 = 0.f;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int a = (NDIM == 3 ? (ly + c / 3) * T::HX : 0) + lx + c % 3;
        const uint4 P = sx[slot][0][a], Q = sx[slot][1][a];
        if (g0) e0 = dot16(P, Q, W5 + 8 * (2 * TZ + c), e0);
        if (g1) e1 = dot16(P, Q, W5 + 8 * (TZ + c), e1);
        if (g2) e2 = dot16(P, Q, W5 + 8 * c, e2);
      }
      a0 += e0;
      a1 += e1;
      a2 += e2;
    }
    if (k - 1 >= k0 && act) {
      const float y = a0 + b0;
      Y[(size_t)(k - 1) * plane + gx + (size_t)d.nx * gy] = scale ? sc * y : y;
    }
    a0 = a1;
    a1 = a2;
    a2 = 0.f;
    if (k < k1) {
      put(slot ^ 1);
      lds_barrier();
      slot ^= 1;
    }
  }
}

template <int NDIM>
int conv5z_tiles(const CnnDims& d) {
  using T = Conv5Z<NDIM>;
  return ((d.nx + T::TX - 1) / T::TX) * (NDIM == 3 ? (d.ny + T::TY - 1) / T::TY : 1) *
         ((d.nz + T::KC - 1) / T::KC);
}

template <int NDIM, int CIN>
int conv_tiles(const CnnDims& d) {
  using T = ConvTile<NDIM, CIN, 0>;
  const int ntx = (d.nx + T::TX - 1) / T::TX;
  const int nty = NDIM == 3 ? (d.ny + T::TY - 1) / T::TY : 1;
  const int ntz = (d.nz + T::TZ - 1) / T::TZ;
  return ntx * nty * ntz;
}

// Weight gradient partials: part[split][co][n] = sum over the split's cells
// p of dY[p][co] * X[p + off(tap(n))][ci(n)], n = tap*CIN + ci.
template <int NDIM, int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad(CnnDims d, const bf16_t* __restrict__ X,
                                               const bf16_t* __restrict__ dY,
                                               float* __restrict__ part) {
  constexpr int NT = Taps<NDIM>::n;
  constexpr int KPAD = (NT * CIN + 31) / 32 * 32;
  constexpr int MTI = COUT / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int n0 = (blockIdx.x * 4 + wave) * 16;
  if (n0 >= KPAD) return;  // no workgroup barrier below
  const int split = blockIdx.y;
  const int p_beg = split * kPixPerSplit;
  const int p_end = min(p_beg + kPixPerSplit, d.npix);
  const int n = n0 + r;
  const int t = n / CIN, ci = n % CIN;
  f32x4 acc[MTI];
#pragma unroll
  for (int mt = 0; mt < MTI; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int p0 = p_beg; p0 < p_end; p0 += 32) {
    bf16x8 b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int p = p0 + 8 * g + i;
      bf16_t v = 0;
      if (p < p_end && t < NT) {
        int a, bb, c;
        coords<NDIM>(d, p, a, bb, c);
        const int q = neighbor<NDIM>(d, a, bb, c, t);
        if (q >= 0) v = X[(size_t)q * CIN + ci];
      }
      b[i] = __builtin_bit_cast(__bf16, v);
    }
#pragma unroll
    for (int mt = 0; mt < MTI; ++mt) {
      bf16x8 a;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int p = p0 + 8 * g + i;
        const bf16_t v = p < p_end ? dY[(size_t)p * COUT + mt * 16 + r] : (bf16_t)0;
        a[i] = __builtin_bit_cast(__bf16, v);
      }
      acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int mt = 0; mt < MTI; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = mt * 16 + 4 * g + i;
      part[((size_t)split * COUT + co) * KPAD + n0 + r] = acc[mt][i];
    }
}

// Sum the weight-gradient partials in split order into the packed gradient
// (logical layout W[co][tap][ci]); the bias gradient sums dY over the cells.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int nsplit,
                                                      int cout_p, int kpad, int cin, int cin_p,
                                                      int cout, int ntaps, float* __restrict__ gW,
                                                      int accumulate) {
  const int total = cout * ntaps * cin;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int ci = e % cin, t = (e / cin) % ntaps, co = e / (cin * ntaps);
    const int n = t * cin_p + ci;
    float s = 0.f;
    for (int sp = 0; sp < nsplit; ++sp) s += part[((size_t)sp * cout_p + co) * kpad + n];
    gW[e] = accumulate ? gW[e] + s : s;
  }
}

// one workgroup per output channel: db[co] = sum_p dY[p][co] (bf16 dY)
__global__ __launch_bounds__(256) void k_bias_grad(const bf16_t* __restrict__ dY, int npix,
                                                   int cout_p, float* __restrict__ gb,
                                                   int accumulate) {
  __shared__ double sh[1][kBlock / 64];
  const int co = blockIdx.x;
  double a[1] = {0.0};
  for (int p = threadIdx.x; p < npix; p += kBlock) a[0] += (double)bf2f(dY[(size_t)p * cout_p + co]);
  Reducer<0u, 1>::block(a, sh);
  if (threadIdx.x == 0) gb[co] = accumulate ? gb[co] + (float)a[0] : (float)a[0];
}

// 2x average pooling (bf16 in and out, FP32 sum); d is the coarse grid
template <int NDIM>
__global__ __launch_bounds__(256) void k_pool(CnnDims d, int C, const bf16_t* __restrict__ X,
                                              bf16_t* __restrict__ Y) {
  const int nxf = 2 * d.nx, nyf = NDIM == 3 ? 2 * d.ny : 1;
  const long total = (long)d.npix * C;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C), q = (int)(e / C);
    int i, j, k;
    coords<NDIM>(d, q, i, j, k);
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < (NDIM == 3 ? 2 : 1); ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int p = (2 * i + dx) + nxf * ((NDIM == 3 ? 2 * j + dy : 0) + nyf * (2 * k + dz));
          s += bf2f(X[(size_t)p * C + c]);
        }
    Y[e] = f2bf(s * (NDIM == 3 ? 0.125f : 0.25f));
  }
}

// Y[p] = [up(A)[p], B[p]] on the fine grid d (A has CA channels, B has CB)
template <int NDIM>
__global__ __launch_bounds__(256) void k_upcat(CnnDims d, int CA, int CB,
                                               const bf16_t* __restrict__ A,
                                               const bf16_t* __restrict__ B,
                                               bf16_t* __restrict__ Y) {
  const int C = CA + CB;
  const int nxc = d.nx / 2, nyc = NDIM == 3 ? d.ny / 2 : 1;
  const long total = (long)d.npix * C;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C), p = (int)(e / C);
    if (c < CA) {
      int i, j, k;
      coords<NDIM>(d, p, i, j, k);
      const int q = (i / 2) + nxc * ((NDIM == 3 ? j / 2 : 0) + nyc * (k / 2));
      Y[e] = A[(size_t)q * CA + c];
    } else {
      Y[e] = B[(size_t)p * CB + (c - CA)];
    }
  }
}

// out = bf16(dy * (y > 0)) (mask = 0: no mask); C channels, padded to Cp in out
__global__ __launch_bounds__(256) void k_mask(int npix, int C, int Cp, const float* __restrict__ dy,
                                              const bf16_t* __restrict__ y, int mask,
                                              bf16_t* __restrict__ out) {
  const long total = (long)npix * Cp;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % Cp), p = (int)(e / Cp);
    float v = 0.f;
    if (c < C) {
      v = dy[(size_t)p * C + c];
      if (mask && !(bf2f(y[(size_t)p * C + c]) > 0.f)) v = 0.f;
    }
    out[e] = f2bf(v);
  }
}

// dA[q] = sum over the fine children of dcat[child][0:CA]; dB[p] = dcat[p][CA:]
template <int NDIM>
__global__ __launch_bounds__(256) void k_upcat_bwd(CnnDims dc, int CA, int CB,
                                                   const float* __restrict__ dcat,
                                                   float* __restrict__ dA, float* __restrict__ dB) {
  const int C = CA + CB;
  const int nxf = 2 * dc.nx, nyf = NDIM == 3 ? 2 * dc.ny : 1;
  const long tA = (long)dc.npix * CA;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tA; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % CA), q = (int)(e / CA);
    int i, j, k;
    coords<NDIM>(dc, q, i, j, k);
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < (NDIM == 3 ? 2 : 1); ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int p = (2 * i + dx) + nxf * ((NDIM == 3 ? 2 * j + dy : 0) + nyf * (2 * k + dz));
          s += dcat[(size_t)p * C + c];
        }
    dA[e] = s;
  }
  const long nfine = (long)dc.npix * (NDIM == 3 ? 8 : 4);
  const long tB = nfine * CB;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tB; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % CB), p = (int)(e / CB);
    dB[e] = dcat[(size_t)p * C + CA + c];
  }
}

// dE[p] += dP[parent(p)] / 2^ndim on the fine grid d
template <int NDIM>
__global__ __launch_bounds__(256) void k_pool_bwd_add(CnnDims d, int C, const float* __restrict__ dP,
                                                      float* __restrict__ dE) {
  const int nxc = d.nx / 2, nyc = NDIM == 3 ? d.ny / 2 : 1;
  const long total = (long)d.npix * C;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C), p = (int)(e / C);
    int i, j, k;
    coords<NDIM>(d, p, i, j, k);
    const int q = (i / 2) + nxc * ((NDIM == 3 ? j / 2 : 0) + nyc * (k / 2));
    dE[e] += dP[(size_t)q * C + c] * (NDIM == 3 ? 0.125f : 0.25f);
  }
}

// dY[p] = (y - t)/npix in channel 0 of 16; loss partials sum (y - t)^2
__global__ __launch_bounds__(256) void k_loss(int npix, const float* __restrict__ y,
                                              const float* __restrict__ t, float* __restrict__ dY,
                                              double* __restrict__ lpart) {
  __shared__ double sh[1][kBlock / 64];
  double a[1] = {0.0};
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += gridDim.x * blockDim.x) {
    const float e = y[p] - t[p];
    dY[p] = e / (float)npix;
    a[0] += (double)e * (double)e;
  }
  Reducer<0u, 1>::block(a, sh);
  if (threadIdx.x == 0) lpart[blockIdx.x] = a[0];
}

// the network input of a cell: x2 (2 channels, what layer 0 reads) and, in
// training instances, xin (the same padded to 8 channels, for the weight
// gradients of layer 0)
__device__ __forceinline__ void put_input(int p, float a, float b, uint32_t* __restrict__ x2,
                                          bf16_t* __restrict__ xin) {
  const bf16_t ha = f2bf(a), hb = f2bf(b);
  x2[p] = (uint32_t)ha | ((uint32_t)hb << 16);
  if (xin) {
    bf16_t* o = xin + (size_t)p * 8;
    o[0] = ha;
    o[1] = hb;
    for (int c = 2; c < 8; ++c) o[c] = 0;
  }
}

__global__ __launch_bounds__(256) void k_input_f32(int npix, const float* __restrict__ xf,
                                                   uint32_t* __restrict__ x2, bf16_t* __restrict__ xin) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += gridDim.x * blockDim.x)
    put_input(p, xf[2 * p], xf[2 * p + 1], x2, xin);
}

__global__ __launch_bounds__(256) void k_input_residual(int npix, const float* __restrict__ r,
                                                        const double* __restrict__ inv_s,
                                                        const float* __restrict__ c,
                                                        const float* __restrict__ dinv,
                                                        uint32_t* __restrict__ x2,
                                                        bf16_t* __restrict__ xin) {
  const float is = (float)*inv_s;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += gridDim.x * blockDim.x)
    put_input(p, r[p] * is, c[p] * dinv[p], x2, xin);
}

// master FP32 (W[co][t][ci], b) -> bf16 W[co_p][kpad] (k = t*cin_p + ci),
// bf16 Wt[ci_p][kpad_t] (k' = flip(t)*cout_p + co), FP32 bias[co_p]
__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ mW, const float* __restrict__ mb,
                                              int cin, int cout, int cin_p, int cout_p, int kpad,
                                              int kpad_t, int cin_t_p, int ntaps,
                                              bf16_t* __restrict__ W, bf16_t* __restrict__ Wt,
                                              float* __restrict__ bias) {
  const long nW = (long)cout_p * kpad;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nW; e += (long)gridDim.x * blockDim.x) {
    const int co = (int)(e / kpad), k = (int)(e % kpad);
    const int t = k / cin_p, ci = k % cin_p;
    float v = 0.f;
    if (co < cout && t < ntaps && ci < cin) v = mW[((long)co * ntaps + t) * cin + ci];
    W[e] = f2bf(v);
  }
  if (Wt) {
    const long nT = (long)cin_t_p * kpad_t;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nT; e += (long)gridDim.x * blockDim.x) {
      const int ci = (int)(e / kpad_t), k = (int)(e % kpad_t);
      const int tf = k / cout_p, co = k % cout_p;
      float v = 0.f;
      if (ci < cin && tf < ntaps && co < cout) {
        const int t = ntaps - 1 - tf;
        v = mW[((long)co * ntaps + t) * cin + ci];
      }
      Wt[e] = f2bf(v);
    }
  }
  for (int co = blockIdx.x * blockDim.x + threadIdx.x; co < cout_p; co += gridDim.x * blockDim.x)
    bias[co] = co < cout ? mb[co] : 0.f;
}

// layer 5: master W[0][t][c] (1 output channel) -> bf16 W5[t][c], taps padded to 32
__global__ __launch_bounds__(256) void k_pack5(const float* __restrict__ mW, int ntaps,
                                               bf16_t* __restrict__ W5) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 32 * 16; e += gridDim.x * blockDim.x) {
    const int t = e / 16, c = e % 16;
    W5[e] = f2bf(t < ntaps ? mW[t * 16 + c] : 0.f);
  }
}

__global__ __launch_bounds__(256) void k_adam(long n, float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr,
                                              float scale, float bc1, float bc2) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const float gr = g[e] * scale;
    const float mm = 0.9f * m[e] + 0.1f * gr;
    const float vv = 0.999f * v[e] + 0.001f * gr * gr;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
  }
}

int blocks_for(long n) {
  long b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

// ---- 3D convolutions as a z-march -----------------------------------------------

// Bias, ReLU and bf16 of RY output rows (16 cells x one 16-channel tile each,
// in MFMA D layout) through a wave's 1 KB LDS scratch: two rows per round,
// then 16 bytes per lane to the channels-last output (COUT channels per cell).
// (kept, when given, receives the lane's bf16 outputs: [row][x] of its channel)
template <int RY, int COUT>
__device__ __forceinline__ void store_rows(const f32x4 (&acc)[RY], float bz, unsigned char* scr,
                                           const CnnDims& d, int x0, int y, int zo, int nt,
                                           bf16_t* __restrict__ Y, bf16_t (*kept)[4] = nullptr) {
  const int lane = threadIdx.x & 63, m = lane & 15, g = lane >> 4;
#pragma unroll
  for (int j0 = 0; j0 < RY; j0 += 2) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bf16_t v = f2bf(fmaxf(acc[j0 + t][i] + bz, 0.f));
        reinterpret_cast<bf16_t*>(scr)[(t * 16 + 4 * g + i) * 16 + m] = v;
        if (kept) kept[j0 + t][i] = v;
      }
    const int t = lane >> 5, cell = (lane >> 1) & 15, c8 = nt * 16 + (lane & 1) * 8;
    const uint4 val = *reinterpret_cast<const uint4*>(scr + lane * 16);
    const int x = x0 + cell, yy = y + j0 + t;
    if (x < d.nx && yy < d.ny)
      *reinterpret_cast<uint4*>(Y + (((size_t)zo * d.ny + yy) * d.nx + x) * COUT + c8) = val;
  }
}

//
// Layers 1, 3 and 4 in 3D; layers 3 and 4 read [up(A), X] (A on the grid one
// level coarser; CA = 0: input X alone).  Here an M
// tile is one output row (16 consecutive x cells at one y, z) and K runs, for
// one input row, over the three x taps and the input channels
// (k = (dx + 1) CIN + channel, padded to a multiple of 32).  A wave owns RY
// output rows and marches through z: each input plane is staged once in LDS
// (fine cells of X and, separately, the coarse cells of A under them), and
// each A operand -- one input row, one 32-wide K chunk -- is read once and
// used for up to nine MFMAs: the three y taps of the output rows it borders
// times the three z taps of the output planes it borders, with accumulators
// for the planes z - 1, z, z + 1.  An output plane is complete once the plane
// above it has been added; it then takes bias and ReLU and leaves through a
// per-wave LDS scratch as 16-byte stores.  The B operands (the weights of one
// K chunk and one (dy, dz) tap pair, prepacked per lane) are read from LDS
// when they fit there, else from global memory.  Each wave computes one 16-channel
// tile of the output channels: with 32 outputs, waves 0-1 and 2-3 take the
// same rows for the two channel tiles.
template <int CIN, int CA, int COUT, int KCH>
struct ConvZ {
  static constexpr int RY = 4;                        // output rows per wave
  static constexpr int NT = COUT / 16;                // output channel tiles
  static constexpr int WG = 4 / NT;                   // waves per channel tile, stacked in y
  static constexpr int TX = 16, TY = WG * RY;         // workgroup tile
  static constexpr int KC = KCH;                      // output planes per workgroup
  static constexpr int CF = CIN - CA;                 // fine channels
  static constexpr int NCH = (3 * CIN + 31) / 32;     // K chunks of one input row
  static constexpr int HX = TX + 2, HY = TY + 2;      // staged fine plane (one-cell halo)
  static constexpr int CHX = TX / 2 + 2, CHY = TY / 2 + 2;  // coarse cells under it
  static constexpr int FROW = HX * CF * 2, CROW = CHX * CA * 2;  // bytes per staged row
  static constexpr int F_OFF = 0, C_OFF = HY * FROW;
  static constexpr int NB = NCH * 9 * NT;             // B fragments, 1 KB each
  static constexpr bool BL = NB * 1024 <= 48 * 1024;  // B in LDS
  static constexpr int B_OFF = C_OFF + CHY * CROW;
  static constexpr int S_OFF = B_OFF + (BL ? NB * 1024 : 0);
  static constexpr int LDS = S_OFF + 4 * 1024;        // + 1 KB output scratch per wave
  static constexpr int FU = HX * HY * (CF / 8), CU = CHX * CHY * (CA / 8);  // 16-byte units per plane
  static constexpr int NL = (FU + CU + 255) / 256;
  static_assert(CF % 8 == 0 && CA % 8 == 0 && COUT % 16 == 0 && COUT <= 64, "layout");
};

template <int CIN, int CA, int COUT, int KCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_z(
    CnnDims d, CnnDims dc, const bf16_t* __restrict__ X,
                                                const bf16_t* __restrict__ A,
                                                const bf16_t* __restrict__ Wz,
                                                const float* __restrict__ bias,
                                                bf16_t* __restrict__ Y) {
  using T = ConvZ<CIN, CA, COUT, KCH>;
  constexpr int RY = T::RY, NT = T::NT, NCH = T::NCH;
  __shared__ __attribute__((aligned(16))) unsigned char sm[T::LDS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, g = lane >> 4;
  const int nt = wave / T::WG, rw = wave % T::WG;  // channel tile, row group
  const int ntx = (d.nx + T::TX - 1) / T::TX, nty = (d.ny + T::TY - 1) / T::TY;
  const int b = xcd_block();
  const int x0 = (b % ntx) * T::TX, y0 = ((b / ntx) % nty) * T::TY;
  const int k0 = (b / (ntx * nty)) * T::KC, k1 = min(k0 + T::KC, d.nz);
  const int cx0 = (x0 - 1) >> 1, cy0 = (y0 - 1) >> 1;  // coarse origin of the staged plane
  if constexpr (T::BL)
    for (int e = threadIdx.x; e < T::NB * 64; e += 256)
      *reinterpret_cast<uint4*>(sm + T::B_OFF + e * 16) = *reinterpret_cast<const uint4*>(Wz + (size_t)e * 8);
  // staging of input plane z: fine cells of X, then the coarse cells of A
  uint4 v[T::NL];
  auto fetch = [&](int z) {
    const bool zin = z >= 0 && z < d.nz;
    const int cz = z >> 1;
#pragma unroll
    for (int u = 0; u < T::NL; ++u) {
      const int e = threadIdx.x + 256 * u;
      v[u] = make_uint4(0, 0, 0, 0);
      if (zin && e < T::FU) {
        const int cell = e / (T::CF / 8), part = e % (T::CF / 8);
        const int x = x0 + cell % T::HX - 1, y = y0 + cell / T::HX - 1;
        if (x >= 0 && x < d.nx && y >= 0 && y < d.ny)
          v[u] = *reinterpret_cast<const uint4*>(X + (((size_t)z * d.ny + y) * d.nx + x) * T::CF + part * 8);
      } else if constexpr (CA > 0) {
        if (zin && e < T::FU + T::CU) {
          const int f = e - T::FU;
          const int cell = f / (CA / 8), part = f % (CA / 8);
          const int x = cx0 + cell % T::CHX, y = cy0 + cell / T::CHX;
          if (x >= 0 && x < dc.nx && y >= 0 && y < dc.ny)
            v[u] = *reinterpret_cast<const uint4*>(A + (((size_t)cz * dc.ny + y) * dc.nx + x) * CA + part * 8);
        }
      }
    }
  };
  auto put = [&]() {
#pragma unroll
    for (int u = 0; u < T::NL; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < T::FU + T::CU)
        *reinterpret_cast<uint4*>(sm + (e < T::FU ? T::F_OFF + e * 16 : T::C_OFF + (e - T::FU) * 16)) = v[u];
    }
  };
  // this lane's A operand offset in K chunk c (staged row 0), and whether
  // its channels are coarse ones
  auto kch = [&](int c, int& dx, int& ch) {
    const int k = 32 * c + 8 * g;
    dx = 0;
    ch = 0;  // K padding: any staged value (its B rows are 0)
    if (k < 3 * CIN) {
      dx = k / CIN - 1;
      ch = k % CIN;
    }
  };
  auto aco_of = [&](int c) {
    int dx, ch;
    kch(c, dx, ch);
    return ch < CA;
  };
  auto aoff_of = [&](int c) {
    int dx, ch;
    kch(c, dx, ch);
    return ch < CA ? T::C_OFF + (((x0 + m + dx) >> 1) - cx0) * (CA * 2) + ch * 2
                   : T::F_OFF + (m + dx + 1) * (T::CF * 2) + (ch - CA) * 2;
  };
  int aoff[T::BL ? NCH : 1];
  bool aco[T::BL ? NCH : 1];
  if constexpr (T::BL)
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      aoff[c] = aoff_of(c);
      aco[c] = aco_of(c);
    }
  const float bz = bias[nt * 16 + m];
  f32x4 aM[RY], a0[RY], aP[RY];  // output planes z - 1, z, z + 1
#pragma unroll
  for (int j = 0; j < RY; ++j) aM[j] = a0[j] = aP[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto loadB = [&](int c, int dy, int dz) {
    const int f = ((c * 3 + dy + 1) * 3 + dz + 1) * NT + nt;
    if constexpr (T::BL)
      return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(sm + T::B_OFF + f * 1024 + lane * 16));
    else
      return load8(Wz + (size_t)f * 512 + lane * 8);
  };
  // A operand of input row r (staged fine row RY*rw + r; its coarse row is
  // (hy + 1) / 2) in K chunk c, at this lane's offset in that chunk
  auto loadA = [&](int off, bool co, int r) {
    const int hy = RY * rw + r;
    const int addr = off + (co ? ((hy + 1) >> 1) * T::CROW : hy * T::FROW);
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(sm + addr));
  };
  // the nine MFMAs of one A operand per output row it borders
  auto chunk = [&](int off, bool co, const bf16x8 (&bw)[3][3]) {
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
      const bf16x8 a = loadA(off, co, r);
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int j = r - 1 - dy;  // output row of tap dy
        if (j < 0 || j >= RY) continue;
        aM[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[dy + 1][2], aM[j], 0, 0, 0);
        a0[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[dy + 1][1], a0[j], 0, 0, 0);
        aP[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[dy + 1][0], aP[j], 0, 0, 0);
      }
    }
  };
  auto loadBs = [&](int c, bf16x8 (&bw)[3][3]) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) bw[dy][dz] = loadB(c, dy - 1, dz - 1);
  };
  // all contributions of the staged plane (input rows RY*rw - 1 ... RY*rw + RY)
  auto compute = [&]() {
    if constexpr (T::BL) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        bf16x8 bw[3][3];
        loadBs(c, bw);
        chunk(aoff[c], aco[c], bw);
      }
    } else {
      // weights from global memory: a rolled loop over chunk pairs, the next
      // chunk's nine B operands in flight during the current chunk
      bf16x8 b0[3][3], b1[3][3];
      loadBs(0, b0);
#pragma unroll 1
      for (int c = 0; c < NCH; c += 2) {
        if (c + 1 < NCH) loadBs(c + 1, b1);
        chunk(aoff_of(c), aco_of(c), b0);
        if (c + 1 < NCH) {
          if (c + 2 < NCH) loadBs(c + 2, b0);
          chunk(aoff_of(c + 1), aco_of(c + 1), b1);
        }
      }
    }
  };
  auto store = [&](int zo) {
    store_rows<RY, COUT>(aM, bz, sm + T::S_OFF + wave * 1024, d, x0, y0 + RY * rw, zo, nt, Y);
  };
  fetch(k0 - 1);
  put();
  __syncthreads();
  for (int z = k0 - 1; z <= k1; ++z) {
    if (z < k1) fetch(z + 1);
    if (z >= 0 && z < d.nz) compute();
    if (z - 1 >= k0) store(z - 1);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      aM[j] = a0[j];
      a0[j] = aP[j];
      aP[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    if (z < k1) {
      __syncthreads();  // every wave is done with plane z
      put();
      __syncthreads();
    }
  }
}

template <int CIN, int CA, int COUT, int KCH>
int convz_tiles(const CnnDims& d) {
  using T = ConvZ<CIN, CA, COUT, KCH>;
  return ((d.nx + T::TX - 1) / T::TX) * ((d.ny + T::TY - 1) / T::TY) * ((d.nz + T::KC - 1) / T::KC);
}

// Layer 0 in 3D as a z-march (2 real input channels, 4 bytes per staged cell).
// A wave owns 4 output rows of 16 cells; one MFMA's K covers the nine (dx, dy)
// taps of one z tap: lane group g < 3 holds the three x taps x 2 channels of
// input row dy = g - 1 (k = 8g ... 8g + 5, three 4-byte LDS reads), the rest
// of K is zero.  Each A operand serves the three z taps: MFMAs into the
// accumulators of planes z - 1, z, z + 1.  W0z holds the three B operands.
struct Conv0Z {
  static constexpr int RY = 4, TX = 16, TY = 4 * RY, KC = 32;
  static constexpr int HX = TX + 2, HY = TY + 2, HP = HX * HY;
  static constexpr int NL = (HP + 255) / 256;
};

// With P0 given, the 2x average pooling of the output (what the next level
// reads) is formed here too, from the same bf16 values in the same order as
// the pooling kernel: each lane holds two x pairs of its channel in the rows
// of its y pairs, and the planes of a z pair come one after the other.
template <bool POOL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_conv0z(CnnDims d, const uint32_t* __restrict__ X2,
                                                const bf16_t* __restrict__ W0z,
                                                const float* __restrict__ bias,
                                                bf16_t* __restrict__ Y, bf16_t* __restrict__ P0) {
  using T = Conv0Z;
  constexpr int RY = T::RY;
  __shared__ uint32_t s2[2][T::HP];  // two planes: the next one is staged while one is read
  __shared__ __attribute__((aligned(16))) unsigned char scr[4 * 1024];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, g = lane >> 4;
  const int ntx = (d.nx + T::TX - 1) / T::TX, nty = (d.ny + T::TY - 1) / T::TY;
  const int b = xcd_block();
  const int x0 = (b % ntx) * T::TX, y0 = ((b / ntx) % nty) * T::TY;
  const int k0 = (b / (ntx * nty)) * T::KC, k1 = min(k0 + T::KC, d.nz);
  bf16x8 bw[3];  // dz = -1, 0, +1
#pragma unroll
  for (int i = 0; i < 3; ++i) bw[i] = load8(W0z + (size_t)(i * 64 + lane) * 8);
  const float bz = bias[m];
  uint32_t v[T::NL];
  // plane z with its halo, zeros outside the grid: every load is made, from
  // an index clamped into the grid, and the zero padding is a select
  auto fetch = [&](int z) {
    const bool zin = z >= 0 && z < d.nz;
    const int zc = z < 0 ? 0 : (z >= d.nz ? d.nz - 1 : z);
#pragma unroll
    for (int u = 0; u < T::NL; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int x = x0 + e % T::HX - 1, y = y0 + e / T::HX - 1;
      const bool in = zin && e < T::HP && x >= 0 && x < d.nx && y >= 0 && y < d.ny;
      const int xc = x < 0 ? 0 : (x >= d.nx ? d.nx - 1 : x);
      const int yc = y < 0 ? 0 : (y >= d.ny ? d.ny - 1 : y);
      const uint32_t t = X2[((size_t)zc * d.ny + yc) * d.nx + xc];
      v[u] = in ? t : 0u;
    }
  };
  auto put = [&](int sl) {
#pragma unroll
    for (int u = 0; u < T::NL; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < T::HP) s2[sl][e] = v[u];
    }
  };
  f32x4 aM[RY], a0[RY], aP[RY];
#pragma unroll
  for (int j = 0; j < RY; ++j) aM[j] = a0[j] = aP[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto compute = [&](int sl) {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      uint4 a = make_uint4(0u, 0u, 0u, 0u);
      if (g < 3) {
        const int h = (RY * wave + j + g) * T::HX + m;  // input row y + g - 1, cells x - 1 ... x + 1
        a.x = s2[sl][h];
        a.y = s2[sl][h + 1];
        a.z = s2[sl][h + 2];
      }
      const bf16x8 av = __builtin_bit_cast(bf16x8, a);
      aM[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[2], aM[j], 0, 0, 0);
      a0[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[1], a0[j], 0, 0, 0);
      aP[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[0], aP[j], 0, 0, 0);
    }
  };
  static_assert(RY % 2 == 0 && T::KC % 2 == 0 && T::TX % 4 == 0, "pooling pairs inside a wave");
  float ps[RY / 2][2];  // pooled sums of this lane: [y pair][x pair]
  bf16_t kept[RY][4];   // the lane's bf16 outputs of the plane
  auto pool = [&](int zo) {
    const bool first = ((zo - k0) & 1) == 0;
#pragma unroll
    for (int yp = 0; yp < RY / 2; ++yp)
#pragma unroll
      for (int xp = 0; xp < 2; ++xp) {
        float sum = first ? 0.f : ps[yp][xp];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) sum += bf2f(kept[2 * yp + dy][2 * xp + dx]);
        ps[yp][xp] = sum;
      }
    if (first) return;
    // the wave's RY/2 x 8 coarse cells x 16 channels through its LDS scratch
    // (after the rows of store_rows are out of it) to 16-byte stores
    static_assert(RY / 2 * 8 * 32 <= 1024, "pooled tile fits the wave's scratch");
    bf16_t* sw = reinterpret_cast<bf16_t*>(scr + wave * 1024);
#pragma unroll
    for (int yp = 0; yp < RY / 2; ++yp)
#pragma unroll
      for (int xp = 0; xp < 2; ++xp) sw[(yp * 8 + 2 * g + xp) * 16 + m] = f2bf(ps[yp][xp] * 0.125f);
    if (lane < RY / 2 * 16) {
      const int nx2 = d.nx / 2, ny2 = d.ny / 2;
      const int cell = lane >> 1, yp = cell >> 3, cx = x0 / 2 + (cell & 7), cy = (y0 + RY * wave) / 2 + yp;
      const uint4 val = *reinterpret_cast<const uint4*>(scr + wave * 1024 + lane * 16);
      if (2 * cx < d.nx && 2 * cy < d.ny)
        *reinterpret_cast<uint4*>(P0 + (((size_t)(zo / 2) * ny2 + cy) * nx2 + cx) * 16 + (lane & 1) * 8) = val;
    }
  };
  fetch(k0 - 1);
  put(0);
  lds_barrier();
  int sl = 0;
  for (int z = k0 - 1; z <= k1; ++z) {
    if (z < k1) fetch(z + 1);
    if (z >= 0 && z < d.nz) compute(sl);
    if (z - 1 >= k0) {
      if constexpr (POOL) {
        store_rows<RY, 16>(aM, bz, scr + wave * 1024, d, x0, y0 + RY * wave, z - 1, 0, Y, kept);
        pool(z - 1);
      } else {
        store_rows<RY, 16>(aM, bz, scr + wave * 1024, d, x0, y0 + RY * wave, z - 1, 0, Y);
      }
    }
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      aM[j] = a0[j];
      a0[j] = aP[j];
      aP[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    if (z < k1) {
      // the other buffer was last read a plane ago, before the last barrier
      put(sl ^ 1);
      lds_barrier();
      sl ^= 1;
    }
  }
}

int conv0z_tiles(const CnnDims& d) {
  using T = Conv0Z;
  return ((d.nx + T::TX - 1) / T::TX) * ((d.ny + T::TY - 1) / T::TY) * ((d.nz + T::KC - 1) / T::KC);
}

// layer 0 z-march weights: fragment dz + 1 holds, for lane 16 g + n,
// B[k = 8 g + i][n] = W[n][tap(dx, dy = g - 1, dz)][ch] with i = 2 (dx + 1) + ch
// for g < 3, i < 6; 0 elsewhere
__global__ __launch_bounds__(256) void k_pack0z(const float* __restrict__ mW, int cout,
                                                bf16_t* __restrict__ W0z) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 3 * 64 * 8; e += gridDim.x * blockDim.x) {
    const int i = e % 8, lane = (e / 8) % 64, dz = e / 512 - 1;
    const int g = lane >> 4, n = lane & 15;
    float v = 0.f;
    if (g < 3 && i < 6 && n < cout) {
      const int dx = i / 2 - 1, ch = i % 2, dy = g - 1;
      const int t = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
      v = mW[((long)n * 27 + t) * 2 + ch];
    }
    W0z[e] = f2bf(v);
  }
}

// z-march weights: fragment f = ((c * 3 + dy + 1) * 3 + dz + 1) * NT + nt holds, for lane
// 16 g + n, B[k = 32 c + 8 g + i][out channel 16 nt + n], i = 0..7, where
// k = (dx + 1) cin + ci; 0 beyond 3 cin
__global__ __launch_bounds__(256) void k_packz(const float* __restrict__ mW, int cin, int cout,
                                               int nch, int ntiles, bf16_t* __restrict__ Wz) {
  const long n = (long)nch * 9 * ntiles * 512;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % 8), lane = (int)((e / 8) % 64);
    long f = e / 512;
    const int nt = (int)(f % ntiles);
    f /= ntiles;
    const int dz = (int)(f % 3) - 1;
    f /= 3;
    const int dy = (int)(f % 3) - 1;
    const int c = (int)(f / 3);
    const int k = 32 * c + 8 * (lane >> 4) + i, co = nt * 16 + (lane & 15);
    float v = 0.f;
    if (k < 3 * cin && co < cout) {
      const int dx = k / cin - 1, ci = k % cin;
      const int t = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
      v = mW[((long)co * 27 + t) * cin + ci];
    }
    Wz[e] = f2bf(v);
  }
}

int conv_blocks(int npix) { return (npix + 4 * 16 * kMT - 1) / (4 * 16 * kMT); }

// ---- dispatch -------------------------------------------------------------------

// forward convolution of a layer; layers 3 and 4 read the concatenation
// [up(A), X] directly (A = e2 / d1 on the coarser grid, X = e1 / e0)
template <int NDIM>
void conv_fwd(const Cnn& n, int layer, const bf16_t* X, const bf16_t* A, void* Y,
              bf16_t* pooled = nullptr, const double* scale = nullptr) {
  const CnnLayer& L = n.L[layer];
  const CnnDims& d = n.d[L.level];
  const dim3 bl(256);
  hipStream_t s = n.s;
#define GEA_CONV(CI, CO, CAA)                                                                   \
  hipLaunchKernelGGL((k_conv_t<NDIM, CI, CO, CAA>), dim3(conv_tiles<NDIM, CI>(d)), bl, 0, s, d, X, \
                     A, n.W[layer], n.bias[layer], (bf16_t*)Y)
  switch (layer) {
    case 0:
      if constexpr (NDIM == 3)
      {
        if (pooled)
          hipLaunchKernelGGL(k_conv0z<true>, dim3(conv0z_tiles(d)), bl, 0, s, d, (const uint32_t*)n.x2,
                             n.W0z, n.bias[0], (bf16_t*)Y, pooled);
        else
          hipLaunchKernelGGL(k_conv0z<false>, dim3(conv0z_tiles(d)), bl, 0, s, d, (const uint32_t*)n.x2,
                             n.W0z, n.bias[0], (bf16_t*)Y, pooled);
      }
      else
        hipLaunchKernelGGL((k_conv0<NDIM>), dim3(conv_tiles<NDIM, 8>(d)), bl, 0, s, d,
                           (const uint32_t*)n.x2, n.W0, n.bias[0], (bf16_t*)Y);
      break;
    case 1:
      if constexpr (NDIM == 3)
        hipLaunchKernelGGL((k_conv_z<16, 0, 32, 16>), dim3(convz_tiles<16, 0, 32, 16>(d)), bl, 0, s, d, d,
                           X, X, n.Wz[1], n.bias[1], (bf16_t*)Y);
      else
        GEA_CONV(16, 32, 0);
      break;
    case 2: GEA_CONV(32, 64, 0); break;
    case 3:
      if constexpr (NDIM == 3)
        hipLaunchKernelGGL((k_conv_z<96, 64, 32, 16>), dim3(convz_tiles<96, 64, 32, 16>(d)), bl, 0, s, d,
                           n.d[L.level + 1], X, A, n.Wz[3], n.bias[3], (bf16_t*)Y);
      else
        GEA_CONV(96, 32, 64);
      break;
    case 4:
      if constexpr (NDIM == 3)
        hipLaunchKernelGGL((k_conv_z<48, 32, 16, 64>), dim3(convz_tiles<48, 32, 16, 64>(d)), bl, 0, s, d,
                           n.d[L.level + 1], X, A, n.Wz[4], n.bias[4], (bf16_t*)Y);
      else
        GEA_CONV(48, 16, 32);
      break;
    case 5:
      hipLaunchKernelGGL((k_conv5z<NDIM>), dim3(conv5z_tiles<NDIM>(d)), bl, 0, s, d, X,
                         (const uint32_t*)n.W5, n.bias[5], (float*)Y, scale);
      break;
  }
#undef GEA_CONV
}

// dX (FP32, cin channels) = conv(dYmasked (bf16, cout_p channels), Wt)
template <int NDIM>
void conv_bwd_data(const Cnn& n, int layer, const bf16_t* dYq, float* dX) {
  const CnnLayer& L = n.L[layer];
  const CnnDims& d = n.d[L.level];
  const dim3 gr(conv_blocks(d.npix)), bl(256);
  hipStream_t s = n.s;
#define GEA_CONVT(CI, CO, YS)                                                                   \
  hipLaunchKernelGGL((k_conv<NDIM, CI, CO, 2>), gr, bl, 0, s, d, dYq, n.Wt[layer],            \
                     (const float*)nullptr, (void*)dX, YS, YS)
  switch (layer) {
    case 1: GEA_CONVT(32, 16, 16); break;
    case 2: GEA_CONVT(64, 32, 32); break;
    case 3: GEA_CONVT(32, 96, 96); break;
    case 4: GEA_CONVT(16, 48, 48); break;
    case 5: GEA_CONVT(16, 16, 16); break;
  }
#undef GEA_CONVT
}

template <int NDIM>
void conv_wgrad(const Cnn& n, int layer, const bf16_t* X, const bf16_t* dYq, bool acc) {
  const CnnLayer& L = n.L[layer];
  const CnnDims& d = n.d[L.level];
  const int nsplit = (d.npix + kPixPerSplit - 1) / kPixPerSplit;
  const dim3 gr((L.kpad / 16 + 3) / 4, nsplit), bl(256);
  hipStream_t s = n.s;
#define GEA_WG(CI, CO) hipLaunchKernelGGL((k_wgrad<NDIM, CI, CO>), gr, bl, 0, s, d, X, dYq, n.part)
  switch (layer) {
    case 0: GEA_WG(8, 16); break;
    case 1: GEA_WG(16, 32); break;
    case 2: GEA_WG(32, 64); break;
    case 3: GEA_WG(96, 32); break;
    case 4: GEA_WG(48, 16); break;
    case 5: GEA_WG(16, 16); break;
  }
#undef GEA_WG
  const int ntaps = NDIM == 2 ? 9 : 27;
  const long nW = (long)L.cout * ntaps * L.cin;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(blocks_for(nW)), bl, 0, s, (const float*)n.part, nsplit,
                     L.cout_p, L.kpad, L.cin, L.cin_p, L.cout, ntaps, n.grad + L.woff, (int)acc);
  hipLaunchKernelGGL(k_bias_grad, dim3(L.cout), bl, 0, s, dYq, d.npix, L.cout_p, n.grad + L.boff,
                     (int)acc);
}

// the forward convolution of one layer on the network's own buffers
template <int NDIM>
void conv_layer(Cnn& n, int layer) {
  const bf16_t* none = nullptr;
  switch (layer) {
    case 0:  // in 3D with the pooling of e0 it forms
      conv_fwd<NDIM>(n, 0, n.xin, none, n.e0, NDIM == 3 ? n.p0 : nullptr);
      break;
    case 1: conv_fwd<NDIM>(n, 1, n.p0, none, n.e1); break;
    case 2: conv_fwd<NDIM>(n, 2, n.p1, none, n.e2); break;
    case 3: conv_fwd<NDIM>(n, 3, n.e1, n.e2, n.d1); break;
    case 4: conv_fwd<NDIM>(n, 4, n.e0, n.d1, n.d0); break;
    case 5: conv_fwd<NDIM>(n, 5, n.d0, none, n.y); break;
  }
}

// (with scale given, the output goes to out as (float)*scale times y; y is not stored)
template <int NDIM>
void forward_t(Cnn& n, const double* scale = nullptr, float* out = nullptr) {
  hipStream_t s = n.s;
  const dim3 bl(256);
  conv_layer<NDIM>(n, 0);  // in 3D it also forms p0
  if constexpr (NDIM == 2)
    hipLaunchKernelGGL(k_pool<NDIM>, dim3(blocks_for((long)n.d[1].npix * 16)), bl, 0, s, n.d[1], 16, (const bf16_t*)n.e0, n.p0);
  conv_layer<NDIM>(n, 1);
  hipLaunchKernelGGL(k_pool<NDIM>, dim3(blocks_for((long)n.d[2].npix * 32)), bl, 0, s, n.d[2], 32, (const bf16_t*)n.e1, n.p1);
  conv_layer<NDIM>(n, 2);
  conv_layer<NDIM>(n, 3);
  conv_layer<NDIM>(n, 4);
  if (scale)
    conv_fwd<NDIM>(n, 5, n.d0, nullptr, out, nullptr, scale);
  else
    conv_layer<NDIM>(n, 5);
  if (n.train) {
    // the concatenated inputs of layers 3 and 4, kept for the weight gradients
    hipLaunchKernelGGL(k_upcat<NDIM>, dim3(blocks_for((long)n.d[1].npix * 96)), bl, 0, s, n.d[1], 64, 32, (const bf16_t*)n.e2, (const bf16_t*)n.e1, n.c1);
    hipLaunchKernelGGL(k_upcat<NDIM>, dim3(blocks_for((long)n.d[0].npix * 48)), bl, 0, s, n.d[0], 32, 16, (const bf16_t*)n.d1, (const bf16_t*)n.e0, n.c0);
  }
}

template <int NDIM>
void backward_t(Cnn& n, bool acc) {
  hipStream_t s = n.s;
  const dim3 bl(256);
  const int N0 = n.d[0].npix, N1 = n.d[1].npix, N2 = n.d[2].npix;
  hipLaunchKernelGGL(k_loss, dim3(cnn_loss_partials(n)), bl, 0, s, N0, (const float*)n.y, (const float*)n.t, n.dy5, n.lpart);
  // layer 5 (no ReLU): dY5 has one channel, padded to 16 for the MFMA kernels
  hipLaunchKernelGGL(k_mask, dim3(blocks_for((long)N0 * 16)), bl, 0, s, N0, 1, 16, (const float*)n.dy5, (const bf16_t*)nullptr, 0, n.q5);
  conv_wgrad<NDIM>(n, 5, n.d0, n.q5, acc);
  conv_bwd_data<NDIM>(n, 5, n.q5, n.dd0);
  // layer 4
  hipLaunchKernelGGL(k_mask, dim3(blocks_for((long)N0 * 16)), bl, 0, s, N0, 16, 16, (const float*)n.dd0, (const bf16_t*)n.d0, 1, n.q4);
  conv_wgrad<NDIM>(n, 4, n.c0, n.q4, acc);
  conv_bwd_data<NDIM>(n, 4, n.q4, n.dc0);
  hipLaunchKernelGGL(k_upcat_bwd<NDIM>, dim3(blocks_for((long)N0 * 16)), bl, 0, s, n.d[1], 32, 16, (const float*)n.dc0, n.dd1, n.de0);
  // layer 3
  hipLaunchKernelGGL(k_mask, dim3(blocks_for((long)N1 * 32)), bl, 0, s, N1, 32, 32, (const float*)n.dd1, (const bf16_t*)n.d1, 1, n.q3);
  conv_wgrad<NDIM>(n, 3, n.c1, n.q3, acc);
  conv_bwd_data<NDIM>(n, 3, n.q3, n.dc1);
  hipLaunchKernelGGL(k_upcat_bwd<NDIM>, dim3(blocks_for((long)N1 * 32)), bl, 0, s, n.d[2], 64, 32, (const float*)n.dc1, n.de2, n.de1);
  // layer 2
  hipLaunchKernelGGL(k_mask, dim3(blocks_for((long)N2 * 64)), bl, 0, s, N2, 64, 64, (const float*)n.de2, (const bf16_t*)n.e2, 1, n.q2);
  conv_wgrad<NDIM>(n, 2, n.p1, n.q2, acc);
  conv_bwd_data<NDIM>(n, 2, n.q2, n.dp1);
  hipLaunchKernelGGL(k_pool_bwd_add<NDIM>, dim3(blocks_for((long)N1 * 32)), bl, 0, s, n.d[1], 32, (const float*)n.dp1, n.de1);
  // layer 1
  hipLaunchKernelGGL(k_mask, dim3(blocks_for((long)N1 * 32)), bl, 0, s, N1, 32, 32, (const float*)n.de1, (const bf16_t*)n.e1, 1, n.q1);
  conv_wgrad<NDIM>(n, 1, n.p0, n.q1, acc);
  conv_bwd_data<NDIM>(n, 1, n.q1, n.dp0);
  hipLaunchKernelGGL(k_pool_bwd_add<NDIM>, dim3(blocks_for((long)N0 * 16)), bl, 0, s, n.d[0], 16, (const float*)n.dp0, n.de0);
  // layer 0 (no input gradient needed)
  hipLaunchKernelGGL(k_mask, dim3(blocks_for((long)N0 * 16)), bl, 0, s, N0, 16, 16, (const float*)n.de0, (const bf16_t*)n.e0, 1, n.q0);
  conv_wgrad<NDIM>(n, 0, n.xin, n.q0, acc);
}

}  // namespace

__global__ __launch_bounds__(256) void k_bf16_to_f32(long n, const bf16_t* __restrict__ a,
                                                     float* __restrict__ out) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    out[e] = __uint_as_float((uint32_t)a[e] << 16);
}

int blocks_for_pub(long n) { return blocks_for(n); }

// ---- network geometry and buffers ------------------------------------------------

static void set_layers(Cnn& n, int ndim) {
  const int nt = ndim == 2 ? 9 : 27;
  const int cin[kCnnLayers] = {kCnnInputs, 16, 32, 96, 48, 16};
  const int cout[kCnnLayers] = {16, 32, 64, 32, 16, 1};
  const int level[kCnnLayers] = {0, 1, 2, 1, 0, 0};
  long off = 0;
  for (int l = 0; l < kCnnLayers; ++l) {
    CnnLayer& L = n.L[l];
    L.cin = cin[l];
    L.cout = cout[l];
    L.cin_p = (cin[l] + 7) / 8 * 8;
    L.cout_p = (cout[l] + 15) / 16 * 16;
    L.level = level[l];
    L.kpad = (nt * L.cin_p + 31) / 32 * 32;
    L.kpad_t = (nt * L.cout_p + 31) / 32 * 32;
    L.cin_t_p = (cin[l] + 15) / 16 * 16;
    L.woff = off;
    off += (long)L.cout * nt * L.cin;
    L.boff = off;
    off += L.cout;
  }
  n.nparams = off;
}

long cnn_param_count(int ndim) {
  Cnn n;
  set_layers(n, ndim);
  return n.nparams;
}

bool cnn_dims_ok(int ndim, int nx, int ny, int nz) {
  if (nx < 4 || nz < 4 || nx % 4 || nz % 4) return false;
  if (ndim == 2) return ny == 1;
  return ny >= 4 && ny % 4 == 0;
}

// 1 KB B fragments of a layer's z-march weights
long convz_frags(const CnnLayer& L) { return (long)((3 * L.cin + 31) / 32) * 9 * (L.cout_p / 16); }

size_t cnn_carve(Cnn& n, int ndim, int nx, int ny, int nz, bool train, char* base, size_t off) {
  n.ndim = ndim;
  n.train = train;
  set_layers(n, ndim);
  for (int l = 0; l < 3; ++l) {
    n.d[l].nx = nx >> l;
    n.d[l].ny = ndim == 3 ? (ny >> l) : 1;
    n.d[l].nz = nz >> l;
    n.d[l].npix = n.d[l].nx * n.d[l].ny * n.d[l].nz;
  }
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) & ~size_t(255);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t N0 = n.d[0].npix, N1 = n.d[1].npix, N2 = n.d[2].npix;
  const size_t B2 = sizeof(bf16_t), F4 = sizeof(float);
  n.master = (float*)take(n.nparams * F4);
  for (int l = 0; l < kCnnLayers; ++l) {
    const CnnLayer& L = n.L[l];
    n.W[l] = (bf16_t*)take((size_t)L.cout_p * L.kpad * B2);
    n.Wt[l] = (train && l > 0) ? (bf16_t*)take((size_t)L.cin_t_p * L.kpad_t * B2) : nullptr;
    n.bias[l] = (float*)take((size_t)L.cout_p * F4);
  }
  n.W0 = (bf16_t*)take((size_t)16 * (((ndim == 3 ? 27 : 9) * 2 + 31) / 32 * 32) * B2);
  n.W5 = (bf16_t*)take((size_t)32 * 16 * B2);
  n.W0z = ndim == 3 ? (bf16_t*)take((size_t)3 * 64 * 8 * B2) : nullptr;
  for (int l = 1; l <= 4; ++l)  // 3D layers 1, 3, 4: z-march weights
    n.Wz[l] = (ndim == 3 && l != 2) ? (bf16_t*)take((size_t)convz_frags(n.L[l]) * 512 * B2) : nullptr;
  n.x2 = (uint32_t*)take(N0 * 4);
  n.xin = train ? (bf16_t*)take(N0 * 8 * B2) : nullptr;
  n.xf = (float*)take(N0 * 2 * F4);
  n.e0 = (bf16_t*)take(N0 * 16 * B2);
  n.p0 = (bf16_t*)take(N1 * 16 * B2);
  n.e1 = (bf16_t*)take(N1 * 32 * B2);
  n.p1 = (bf16_t*)take(N2 * 32 * B2);
  n.e2 = (bf16_t*)take(N2 * 64 * B2);
  n.c1 = train ? (bf16_t*)take(N1 * 96 * B2) : nullptr;
  n.d1 = (bf16_t*)take(N1 * 32 * B2);
  n.c0 = train ? (bf16_t*)take(N0 * 48 * B2) : nullptr;
  n.d0 = (bf16_t*)take(N0 * 16 * B2);
  n.y = (float*)take(N0 * F4);
  if (train) {
    n.grad = (float*)take(n.nparams * F4);
    n.m = (float*)take(n.nparams * F4);
    n.v = (float*)take(n.nparams * F4);
    n.t = (float*)take(N0 * F4);
    n.dy5 = (float*)take(N0 * F4);
    n.dd0 = (float*)take(N0 * 16 * F4);
    n.dc0 = (float*)take(N0 * 48 * F4);
    n.dd1 = (float*)take(N1 * 32 * F4);
    n.de0 = (float*)take(N0 * 16 * F4);
    n.dc1 = (float*)take(N1 * 96 * F4);
    n.de2 = (float*)take(N2 * 64 * F4);
    n.de1 = (float*)take(N1 * 32 * F4);
    n.dp1 = (float*)take(N2 * 32 * F4);
    n.dp0 = (float*)take(N1 * 16 * F4);
    n.q5 = (bf16_t*)take(N0 * 16 * B2);
    n.q4 = (bf16_t*)take(N0 * 16 * B2);
    n.q3 = (bf16_t*)take(N1 * 32 * B2);
    n.q2 = (bf16_t*)take(N2 * 64 * B2);
    n.q1 = (bf16_t*)take(N1 * 32 * B2);
    n.q0 = (bf16_t*)take(N0 * 16 * B2);
    long mx = 0;
    for (int l = 0; l < kCnnLayers; ++l) {
      const CnnLayer& L = n.L[l];
      const long ns = (n.d[L.level].npix + kPixPerSplit - 1) / kPixPerSplit;
      const long need = ns * L.cout_p * L.kpad;
      if (need > mx) mx = need;
    }
    n.part_floats = mx;
    n.part = (float*)take((size_t)mx * F4);
    n.lpart = (double*)take(sizeof(double) * 1024);
  }
  return off;
}

int cnn_loss_partials(const Cnn& n) { return blocks_for(n.d[0].npix) > 1024 ? 1024 : blocks_for(n.d[0].npix); }

void cnn_pack_weights(Cnn& n) {
  const int nt = n.ndim == 2 ? 9 : 27;
  hipLaunchKernelGGL(k_pack5, dim3(2), dim3(256), 0, n.s, (const float*)(n.master + n.L[5].woff), nt,
                     n.W5);
  {
    const CnnLayer& L = n.L[0];
    const int kp0 = (nt * 2 + 31) / 32 * 32;
    hipLaunchKernelGGL(k_pack, dim3(blocks_for((long)16 * kp0)), dim3(256), 0, n.s,
                       (const float*)(n.master + L.woff), (const float*)(n.master + L.boff), L.cin,
                       L.cout, 2, 16, kp0, 0, 0, nt, n.W0, (bf16_t*)nullptr, n.bias[0]);
  }
  if (n.W0z)
    hipLaunchKernelGGL(k_pack0z, dim3(2), dim3(256), 0, n.s, (const float*)(n.master + n.L[0].woff),
                       n.L[0].cout, n.W0z);
  for (int l = 1; l <= 4; ++l)
    if (n.Wz[l]) {
      const CnnLayer& L = n.L[l];
      const long work = (long)convz_frags(L) * 512;
      hipLaunchKernelGGL(k_packz, dim3(blocks_for(work)), dim3(256), 0, n.s,
                         (const float*)(n.master + L.woff), L.cin, L.cout, (3 * L.cin + 31) / 32,
                         L.cout_p / 16, n.Wz[l]);
    }
  for (int l = 0; l < kCnnLayers; ++l) {
    const CnnLayer& L = n.L[l];
    const long work = (long)L.cout_p * L.kpad + (long)L.cin_t_p * L.kpad_t;
    hipLaunchKernelGGL(k_pack, dim3(blocks_for(work)), dim3(256), 0, n.s,
                       (const float*)(n.master + L.woff), (const float*)(n.master + L.boff), L.cin,
                       L.cout, L.cin_p, L.cout_p, L.kpad, L.kpad_t, L.cin_t_p, nt, n.W[l],
                       n.Wt[l], n.bias[l]);
  }
}

void cnn_input_from_f32(Cnn& n) {
  hipLaunchKernelGGL(k_input_f32, dim3(blocks_for(n.d[0].npix)), dim3(256), 0, n.s, n.d[0].npix,
                     (const float*)n.xf, n.x2, n.xin);
}

void cnn_input_from_residual(Cnn& n, const float* r, const double* inv_s, const float* c,
                             const float* dinv) {
  hipLaunchKernelGGL(k_input_residual, dim3(blocks_for(n.d[0].npix)), dim3(256), 0, n.s,
                     n.d[0].npix, r, inv_s, c, dinv, n.x2, n.xin);
}


void cnn_forward(Cnn& n) {
  if (n.ndim == 2) forward_t<2>(n);
  else forward_t<3>(n);
}

void cnn_forward_scaled(Cnn& n, const double* s, float* out) {
  if (n.ndim == 2) forward_t<2>(n, s, out);
  else forward_t<3>(n, s, out);
}

void cnn_conv_layer(Cnn& n, int layer) {
  if (n.ndim == 2) conv_layer<2>(n, layer);
  else conv_layer<3>(n, layer);
}

double cnn_layer_flops(const Cnn& n, int layer) {
  const CnnLayer& L = n.L[layer];
  const double taps = n.ndim == 2 ? 9.0 : 27.0;
  return 2.0 * (double)n.d[L.level].npix * L.cout * taps * L.cin;
}

void cnn_backward(Cnn& n, bool accumulate) {
  if (n.ndim == 2) backward_t<2>(n, accumulate);
  else backward_t<3>(n, accumulate);
}

// An activation of the last forward pass as FP32, channels last (see
// gea_cnn_activation for `which`); which = 0 on an inference instance gives
// the two input channels it keeps (r/s, c/diag per cell).
gea_status cnn_copy_activation(Cnn& n, int which, float* out, gea_ptr_kind kind, std::string& err) {
  auto ok = [&](hipError_t e) {
    if (e == hipSuccess) return true;
    err = std::string("HIP error in activation: ") + hipGetErrorString(e);
    return false;
  };
  const hipMemcpyKind dir = kind == GEA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (which == 10) {
    if (!ok(hipMemcpyAsync(out, n.y, sizeof(float) * n.d[0].npix, dir, n.s))) return GEA_ERR_HIP;
    return ok(hipStreamSynchronize(n.s)) ? GEA_OK : GEA_ERR_HIP;
  }
  const bf16_t* src[10] = {n.xin, n.e0, n.p0, n.e1, n.p1, n.e2, n.c1, n.d1, n.c0, n.d0};
  const int lev[10] = {0, 0, 1, 1, 2, 2, 1, 1, 0, 0};
  int ch[10] = {8, 16, 16, 32, 32, 64, 96, 32, 48, 16};
  if (which == 0 && !n.xin) {  // the 2-channel input: each x2 word holds (r/s, c/diag)
    src[0] = reinterpret_cast<const bf16_t*>(n.x2);
    ch[0] = 2;
  }
  if (!src[which]) {
    err = "the concatenated inputs are kept by training instances only";
    return GEA_ERR_STATE;
  }
  const long count = (long)n.d[lev[which]].npix * ch[which];
  // host copies go through the FP32 input staging buffer (2 values a cell)
  const long chunk = 2L * n.d[0].npix;
  for (long off = 0; off < count; off += chunk) {
    const long m = count - off < chunk ? count - off : chunk;
    float* d = kind == GEA_HOST ? n.xf : out + off;
    hipLaunchKernelGGL(k_bf16_to_f32, dim3(blocks_for(m)), dim3(256), 0, n.s, m, src[which] + off, d);
    if (!ok(hipGetLastError())) return GEA_ERR_HIP;
    if (kind == GEA_HOST) {
      if (!ok(hipMemcpyAsync(out + off, n.xf, sizeof(float) * m, hipMemcpyDeviceToHost, n.s))) return GEA_ERR_HIP;
      if (!ok(hipStreamSynchronize(n.s))) return GEA_ERR_HIP;
    }
  }
  return ok(hipStreamSynchronize(n.s)) ? GEA_OK : GEA_ERR_HIP;
}

void cnn_adam(Cnn& n, float lr, float scale, int step) {
  const float bc1 = 1.f - powf(0.9f, (float)step), bc2 = 1.f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n.nparams)), dim3(256), 0, n.s, n.nparams, n.master,
                     (const float*)n.grad, n.m, n.v, lr, scale, bc1, bc2);
  cnn_pack_weights(n);
}

}  // namespace gea

// ---- C ABI -----------------------------------------------------------------------------

struct gea_cnn {
  gea::Cnn net;
  std::string err;
};

namespace {
hipMemcpyKind kin(gea_ptr_kind k) { return k == GEA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
hipMemcpyKind kout(gea_ptr_kind k) { return k == GEA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }
gea_status hip_status(gea_cnn* x, hipError_t e, const char* what) {
  if (e == hipSuccess) return GEA_OK;
  if (x) x->err = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
  return GEA_ERR_HIP;
}
}  // namespace

extern "C" {

gea_status gea_cnn_param_count(int32_t ndim, int64_t* count) {
  if ((ndim != 2 && ndim != 3) || !count) return GEA_ERR_ARG;
  *count = gea::cnn_param_count(ndim);
  return GEA_OK;
}

gea_status gea_cnn_workspace_bytes(int32_t ndim, int32_t nx, int32_t ny, int32_t nz,
                                   int32_t train, size_t* bytes) {
  if ((ndim != 2 && ndim != 3) || !bytes || !gea::cnn_dims_ok(ndim, nx, ny, nz)) return GEA_ERR_ARG;
  if ((double)nx * ny * nz > 1.5e8) return GEA_ERR_ARG;
  gea::Cnn n;
  *bytes = gea::cnn_carve(n, ndim, nx, ny, nz, train != 0, nullptr, 0) + 256;
  return GEA_OK;
}

gea_status gea_cnn_create(int32_t ndim, int32_t nx, int32_t ny, int32_t nz, int32_t train,
                          void* hip_stream, void* workspace, size_t workspace_bytes,
                          gea_cnn** out) {
  if (!out) return GEA_ERR_ARG;
  *out = nullptr;
  size_t need = 0;
  if (gea_cnn_workspace_bytes(ndim, nx, ny, nz, train, &need) != GEA_OK) return GEA_ERR_ARG;
  if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255u))
    return GEA_ERR_ARG;
  gea_cnn* x = new (std::nothrow) gea_cnn();
  if (!x) return GEA_ERR_ALLOC;
  gea::cnn_carve(x->net, ndim, nx, ny, nz, train != 0, static_cast<char*>(workspace), 0);
  x->net.s = static_cast<hipStream_t>(hip_stream);
  *out = x;
  return GEA_OK;
}

gea_status gea_cnn_set_params(gea_cnn* x, const float* params, gea_ptr_kind kind) {
  if (!x || !params) return GEA_ERR_ARG;
  gea::Cnn& n = x->net;
  const size_t bytes = sizeof(float) * n.nparams;
  gea_status st = hip_status(x, hipMemcpyAsync(n.master, params, bytes, kin(kind), n.s), "params");
  if (st != GEA_OK) return st;
  if (n.train) {
    if ((st = hip_status(x, hipMemsetAsync(n.m, 0, bytes, n.s), "m")) != GEA_OK) return st;
    if ((st = hip_status(x, hipMemsetAsync(n.v, 0, bytes, n.s), "v")) != GEA_OK) return st;
    if ((st = hip_status(x, hipMemsetAsync(n.grad, 0, bytes, n.s), "grad")) != GEA_OK) return st;
  }
  gea::cnn_pack_weights(n);
  return hip_status(x, hipStreamSynchronize(n.s), "set_params");
}

gea_status gea_cnn_get_params(gea_cnn* x, float* params, gea_ptr_kind kind) {
  if (!x || !params) return GEA_ERR_ARG;
  gea::Cnn& n = x->net;
  gea_status st = hip_status(x, hipMemcpyAsync(params, n.master, sizeof(float) * n.nparams, kout(kind), n.s), "get_params");
  if (st != GEA_OK) return st;
  return hip_status(x, hipStreamSynchronize(n.s), "get_params");
}

gea_status gea_cnn_forward(gea_cnn* x, const float* in, float* y, gea_ptr_kind kind) {
  if (!x || !in || !y) return GEA_ERR_ARG;
  gea::Cnn& n = x->net;
  const size_t N0 = n.d[0].npix;
  gea_status st = hip_status(x, hipMemcpyAsync(n.xf, in, N0 * 2 * sizeof(float), kin(kind), n.s), "input");
  if (st != GEA_OK) return st;
  gea::cnn_input_from_f32(n);
  gea::cnn_forward(n);
  if ((st = hip_status(x, hipGetLastError(), "forward")) != GEA_OK) return st;
  st = hip_status(x, hipMemcpyAsync(y, n.y, N0 * sizeof(float), kout(kind), n.s), "output");
  if (st != GEA_OK) return st;
  return hip_status(x, hipStreamSynchronize(n.s), "forward");
}

gea_status gea_cnn_backward(gea_cnn* x, const float* target, gea_ptr_kind kind,
                            int32_t accumulate, double* loss) {
  if (!x || !target) return GEA_ERR_ARG;
  gea::Cnn& n = x->net;
  if (!n.train) {
    x->err = "not a training instance";
    return GEA_ERR_STATE;
  }
  const size_t N0 = n.d[0].npix;
  gea_status st = hip_status(x, hipMemcpyAsync(n.t, target, N0 * sizeof(float), kin(kind), n.s), "target");
  if (st != GEA_OK) return st;
  gea::cnn_backward(n, accumulate != 0);
  if ((st = hip_status(x, hipGetLastError(), "backward")) != GEA_OK) return st;
  if (loss) {
    const int np = gea::cnn_loss_partials(n);
    double h[1024];
    st = hip_status(x, hipMemcpyAsync(h, n.lpart, np * sizeof(double), hipMemcpyDeviceToHost, n.s), "loss");
    if (st != GEA_OK) return st;
    if ((st = hip_status(x, hipStreamSynchronize(n.s), "loss")) != GEA_OK) return st;
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += h[i];
    *loss = s / (2.0 * (double)N0);
  }
  return hip_status(x, hipStreamSynchronize(n.s), "backward");
}

gea_status gea_cnn_get_grads(gea_cnn* x, float* grads, gea_ptr_kind kind) {
  if (!x || !grads) return GEA_ERR_ARG;
  gea::Cnn& n = x->net;
  if (!n.train) return GEA_ERR_STATE;
  gea_status st = hip_status(x, hipMemcpyAsync(grads, n.grad, sizeof(float) * n.nparams, kout(kind), n.s), "grads");
  if (st != GEA_OK) return st;
  return hip_status(x, hipStreamSynchronize(n.s), "grads");
}

gea_status gea_cnn_adam(gea_cnn* x, float lr, float grad_scale, int32_t step) {
  if (!x || step < 1 || !(lr > 0)) return GEA_ERR_ARG;
  gea::Cnn& n = x->net;
  if (!n.train) return GEA_ERR_STATE;
  gea::cnn_adam(n, lr, grad_scale, step);
  gea_status st = hip_status(x, hipGetLastError(), "adam");
  if (st != GEA_OK) return st;
  return hip_status(x, hipStreamSynchronize(n.s), "adam");
}

gea_status gea_cnn_activation(gea_cnn* x, int32_t which, float* out, gea_ptr_kind kind) {
  if (!x || !out || which < 0 || which > 10) return GEA_ERR_ARG;
  return gea::cnn_copy_activation(x->net, which, out, kind, x->err);
}

void gea_cnn_destroy(gea_cnn* x) { delete x; }

}  // extern "C"

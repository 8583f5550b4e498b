// Learned warm start: a 3-D convolution network on the periodic grid,
// trained and run by the library's own kernels.
//
// Layout: activations are bf16 [p][24] with p = (x n + y) n + z (z fastest);
// the network input/output and loss gradients are f32 [p].  Every kernel works
// on output tiles (4 x 8 x 8 cells for the vector-ALU layers, 8 x 8 x 8 for the
// matrix-core layers; z fastest) with a one-cell periodic halo staged in LDS.
//
// * 24 -> 24 convolutions run on the matrix cores as an implicit GEMM per
//   tile: D[cell][out] = sum_k A[cell][k] B[k][out], k = (tap, in-channel),
//   with v_mfma_f32_16x16x32_bf16 (16 cells x 32 k x 16 channels per
//   instruction, FP32 accumulation).  K = 27 taps x 24 channels is walked in
//   chunks of 8 channels (one 16-byte LDS read per lane); 81 chunks are padded
//   to 84 (21 MFMA steps); 24 output channels use two 16-wide tiles.  The
//   gradient with respect to the input is the same kernel with transposed,
//   tap-flipped weights.
// * Weight gradients are correlations over all cells,
//   dW[m][n][tap] = sum_p U[p][m] V[p + tap][n]; they run on the matrix cores
//   with the cells as the K dimension (runs of 8 cells along z, pre-shifted
//   copies of V in LDS for the three z offsets), in persistent workgroups that
//   write per-workgroup partial sums, added in a fixed order afterwards.
// * The 24 -> 1 layers (the last layer, and the input gradient of the first)
//   run on the same matrix-core kernel with one 16-wide output tile of which
//   one column is used.  The first layer (1 -> 24) runs on the matrix cores
//   with the 27 taps as K (padded to 32); the input gradient of the last
//   layer (also 1 -> 24, followed by the GELU derivative) uses the vector ALU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "level.h"
#include "../../include/mgnn.h"

namespace mg {
namespace {

typedef uint16_t bf16_t;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kC = 24;                                // hidden channels
constexpr int kTaps = 27;
constexpr int TX = 4, TY = 8, TZ = 8;                 // output tile (cells), z fastest
constexpr int kTile = TX * TY * TZ;                   // 256 cells, one per thread
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;  // tile + one-cell halo
constexpr int kHalo = HX * HY * HZ;                   // 600
constexpr int kChunks = kTaps * 3;                    // K chunks of 8 channels
constexpr int kKSteps = (kChunks + 3) / 4;            // MFMA steps of K = 32
constexpr int kPackVecs = kKSteps * 2 * 64;           // packed B fragments (16 B each)

// flat parameter offsets: W_l then b_l per layer
constexpr int kW0 = 0, kB0 = kW0 + kC * kTaps;
constexpr int kW1 = kB0 + kC;
constexpr int kHiddenBlock = kC * kC * kTaps + kC;
constexpr int kW4 = kW1 + 3 * kHiddenBlock, kB4 = kW4 + kC * kTaps;
constexpr int kNumParams = kB4 + 1;                   // 48049
__host__ __device__ constexpr int w_off(int l) { return l == 0 ? kW0 : (l == 4 ? kW4 : kW1 + (l - 1) * kHiddenBlock); }
__host__ __device__ constexpr int b_off(int l) { return l == 0 ? kB0 : (l == 4 ? kB4 : w_off(l) + kC * kC * kTaps); }

__device__ __forceinline__ bf16_t f2bf(float f) {   // round to nearest even (gfx950's v_cvt_pk_bf16_f32)
  return __builtin_bit_cast(bf16_t, (__bf16)f);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float bfr(float f) { return bf2f(f2bf(f)); }
// GELU by the tanh form of Hendrycks & Gimpel (2016),
// u/2 (1 + tanh(sqrt(2/pi) (u + 0.044715 u^3))) = u sigma(y),
// y = 2 sqrt(2/pi) (u + 0.044715 u^3): one exp2 and one reciprocal.  It
// differs from the exact u/2 (1 + erf(u/sqrt 2)) by at most 4.7e-4 (at
// u = -2.7; the derivative by at most 8.7e-4), below the bfloat16 spacing
// (2^-8) of activations of order 1.  The derivative is that of the same
// form, sigma + u sigma (1 - sigma) y'.
constexpr float kGeluC1 = 1.5957691216057308f;              // 2 sqrt(2/pi)
constexpr float kGeluC3 = 0.071354816272919f;               // 2 sqrt(2/pi) 0.044715
constexpr float kLog2e = 1.4426950408889634f;
__device__ __forceinline__ float gelu_sigma(float u, float& yp) {
  const float u2 = u * u;
  yp = fmaf(3.0f * kGeluC3, u2, kGeluC1);                     // dy/du
  const float ny = u * fmaf(-kGeluC3 * kLog2e, u2, -kGeluC1 * kLog2e);   // -y log2(e)
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(ny));      // sigma(y); 0 when exp2 overflows
}
__device__ __forceinline__ float gelu(float u) {
  float yp;
  return u * gelu_sigma(u, yp);
}
__device__ __forceinline__ float gelu_grad(float u) {
  float yp;
  const float sg = gelu_sigma(u, yp);
  const float d = sg - sg * sg;   // sigma (1 - sigma): 0 where sigma saturates
  return d > 0.0f ? fmaf(u * d, yp, sg) : sg;
}

// two floats -> two bf16 (round to nearest even) in one word, a in the low
// half: one v_cvt_pk_bf16_f32
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t{a, b}), bf16x2_t));
}
// 8 floats -> 8 bf16 (round to nearest even) in one 16-byte word, and back
__device__ __forceinline__ uint4 pack8(const float (&v)[8]) {
  uint4 r;
  r.x = pack2(v[0], v[1]);
  r.y = pack2(v[2], v[3]);
  r.z = pack2(v[4], v[5]);
  r.w = pack2(v[6], v[7]);
  return r;
}
__device__ __forceinline__ void unpack8(uint4 r, float (&v)[8]) {
  v[0] = __uint_as_float(r.x << 16);
  v[1] = __uint_as_float(r.x & 0xFFFF0000u);
  v[2] = __uint_as_float(r.y << 16);
  v[3] = __uint_as_float(r.y & 0xFFFF0000u);
  v[4] = __uint_as_float(r.z << 16);
  v[5] = __uint_as_float(r.z & 0xFFFF0000u);
  v[6] = __uint_as_float(r.w << 16);
  v[7] = __uint_as_float(r.w & 0xFFFF0000u);
}

__device__ __forceinline__ int64_t didx(int x, int y, int z, int m, int lg) {
  return ((int64_t)(x & m) << (2 * lg)) | ((int64_t)(y & m) << lg) | (int64_t)(z & m);
}
__device__ __forceinline__ void tap_offset(int t, int& dx, int& dy, int& dz) {
  dx = t / 9 - 1;
  dy = (t / 3) % 3 - 1;
  dz = t % 3 - 1;
}

// tile origin of workgroup `bid` (XCD-aware order when the tile count allows)
__device__ __forceinline__ void tile_origin(int lg, int bid, int& x0, int& y0, int& z0) {
  const int n = 1 << lg;
  const int tnx = n / TX, tny = n / TY, tnz = n / TZ;
  const int count = tnx * tny * tnz;
  int t = bid;
  if ((count & 7) == 0 && (int)gridDim.x == count) t = (bid & 7) * (count >> 3) + (bid >> 3);
  z0 = (t % tnz) * TZ;
  y0 = ((t / tnz) % tny) * TY;
  x0 = (t / (tnz * tny)) * TX;
}

__device__ __forceinline__ void tile_cell(int c, int& mx, int& my, int& mz) {
  mx = c / (TY * TZ);
  my = (c / TZ) % TY;
  mz = c % TZ;
}
__device__ __forceinline__ int halo_cell(int hx, int hy, int hz) { return (hx * HY + hy) * HZ + hz; }

// ---------------------------------------------------------------------------
// 24 -> 24 convolution on the matrix cores
//   MODE 0 (forward): z = conv + bias; stores z (if out_z) and a = gelu(z), bf16
//   MODE 1 (input gradient): g = conv(dz_next, W^T flipped) * gelu'(zprev) -> out_z
// ---------------------------------------------------------------------------
// tiles of the matrix-core convolution: 8 x 8 x 8 cells, four waves of eight
// 16-cell M-tiles each; the halo (10^3 cells x 24 channels, bf16) and then the
// f32 output staging share one LDS buffer
constexpr int QX = 8, QY = 8, QZ = 8, kQTile = QX * QY * QZ;        // 512 cells
constexpr int QHX = QX + 2, QHY = QY + 2, QHZ = QZ + 2, kQHalo = QHX * QHY * QHZ;   // 1000
constexpr int kQShared = kQTile * kC * 4;                           // f32 staging of the outputs (49152 B)
static_assert(kQHalo * kC * 2 <= kQShared, "halo tile fits the shared buffer");
// Cells of M tile t (0..31) of the 8 x 8 x 8 output tile: rows 0..7 are the z
// line (x, y), rows 8..15 the z line (x, y + 4), x = t / 4, y = t % 4.  Two
// z lines 4 apart start 4 x 10 x 48 B = 1920 B apart in the halo box, which
// is 128 B modulo the 256 B the LDS banks span: the 16-byte A-fragment reads
// of a row group (16 cells, 48 B apart) then fall on 16 distinct bank
// quadruples (adjacent lines, 480 B apart, made two of them collide).
__device__ __forceinline__ void qcell(int t, int row, int& mx, int& my, int& mz) {
  mx = t >> 2;
  my = (t & 3) + ((row >> 3) << 2);
  mz = row & 7;
}

// tile t: z fastest, so consecutive tiles share their z faces
__device__ __forceinline__ void qtile_origin(int lg, int t, int& x0, int& y0, int& z0) {
  const int n = 1 << lg;
  const int tny = n / QY, tnz = n / QZ;
  z0 = (t % tnz) * QZ;
  y0 = ((t / tnz) % tny) * QY;
  x0 = (t / (tnz * tny)) * QX;
}

// The halo box of a tile ([p][24] bf16, QHX x QHY x QHZ cells with lower
// corner (x0 - 1, y0 - 1, z0 - 1)) in 16-byte pieces: loaded into registers
// (all loads in flight together), later stored to LDS as s[cell][24].
constexpr int kQBoxVec = kQHalo * 3;
constexpr int kQBoxPer = (kQBoxVec + 255) / 256;
// (a native vector type: the HIP uint4 struct is copied through memory)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void qbox_load(const bf16_t* __restrict__ in, int x0, int y0, int z0, int m, int lg,
                                          u32x4 (&v)[kQBoxPer]) {
#pragma unroll
  for (int r = 0; r < kQBoxPer; ++r) {
    const int q = min((int)threadIdx.x + r * 256, kQBoxVec - 1);
    const int cell = q / 3, part = q % 3;
    const int hx = cell / (QHY * QHZ), hy = (cell / QHZ) % QHY, hz = cell % QHZ;
    v[r] = *reinterpret_cast<const u32x4*>(in + didx(x0 - 1 + hx, y0 - 1 + hy, z0 - 1 + hz, m, lg) * kC + part * 8);
  }
}
__device__ __forceinline__ void qbox_store(bf16_t* s, const u32x4 (&v)[kQBoxPer]) {
#pragma unroll
  for (int r = 0; r < kQBoxPer; ++r) {
    const int q = threadIdx.x + r * 256;
    if (q < kQBoxVec) *reinterpret_cast<u32x4*>(s + q * 8) = v[r];   // cell * 24 + part * 8 = 8 q
  }
}

//   MODE 2 (24 -> 1, one N tile): y = conv + bias (if bias) -> out1 (f32); the
//   last layer, and the input gradient of the first layer (transposed weights)
// Persistent: two workgroups per CU for the 24 -> 24 layers, three for the
// 24 -> 1 ones (one LDS buffer of kQShared bytes each; the register budget
// holds the next tile's box besides the accumulators), each taking a
// contiguous run of tiles.  The next tile's halo box is
// loaded into registers after this tile's matrix products and stored into
// the buffer after the epilogue has read its outputs back, so the box loads
// run behind the epilogue instead of in front of the products.
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == 2 ? 3 : 2))) void k_conv24(int lg, int n_tiles, const bf16_t* __restrict__ in,
                                                const uint4* __restrict__ wpk,
                                                const float* __restrict__ bias, const bf16_t* __restrict__ zprev,
                                                bf16_t* __restrict__ out_z, bf16_t* __restrict__ out_a,
                                                float* __restrict__ out1) {
  constexpr int NT = MODE == 2 ? 1 : 2;      // 16-wide output tiles
  __shared__ __attribute__((aligned(16))) unsigned char q_lds[kQShared];
  __shared__ int s_off[kKSteps * 4];   // byte offset of K chunk j's inputs from a cell's own (tap, channels)
  const int m = (1 << lg) - 1;
  const int per = n_tiles / (int)gridDim.x, extra = n_tiles % (int)gridDim.x;
  const int t_begin = (int)blockIdx.x * per + min((int)blockIdx.x, extra);
  const int t_end = t_begin + per + ((int)blockIdx.x < extra ? 1 : 0);
  int x0, y0, z0;
  qtile_origin(lg, t_begin, x0, y0, z0);
  {
    u32x4 first[kQBoxPer];
    qbox_load(in, x0, y0, z0, m, lg, first);
    qbox_store(reinterpret_cast<bf16_t*>(q_lds), first);
  }
  if (threadIdx.x < kKSteps * 4) {
    // the padding chunks (81..83, zero weights) read chunk 0's inputs: finite values
    const int j = (int)threadIdx.x < kChunks ? (int)threadIdx.x : 0;
    int dx, dy, dz;
    tap_offset(j / 3, dx, dy, dz);
    s_off[threadIdx.x] = (((dx * QHY + dy) * QHZ + dz) * kC + (j % 3) * 8) * 2;
  }
  // this lane's output-channel biases, read once (a global load inside the
  // epilogue would wait for the next box's loads)
  float bias_reg[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int o = nt * 16 + ((int)threadIdx.x & 15);
    bias_reg[nt] = MODE == 0 ? (o < kC ? bias[o] : 0.f) : (MODE == 2 && bias ? bias[0] : 0.f);
  }
  __syncthreads();

  for (int t = t_begin, it = 0; t < t_end; ++t, ++it) {
  bf16_t* s = reinterpret_cast<bf16_t*>(q_lds);
  const bool has_next = t + 1 < t_end;
  int nx0, ny0, nz0;
  qtile_origin(lg, has_next ? t + 1 : t, nx0, ny0, nz0);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row = l & 15, kb = l >> 4;
  constexpr int MT = kQTile / 16 / 4;         // M-tiles (16 cells) per wave: 8
  f32x4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  // this lane's row in the wave's first M tile; M tile mt (tile t = 8 w + mt:
  // x = 2 w + mt / 4, y = mt % 4 (+ 4 for rows 8..15)) lies a compile-time
  // distance further, which goes into the LDS loads' offset field
  int hc0;
  {
    int mx, my, mz;
    qcell(w * MT, row, mx, my, mz);
    hc0 = (((mx + 1) * QHY) + (my + 1)) * QHZ + (mz + 1);
  }
  const char* sb = reinterpret_cast<const char*>(s) + hc0 * kC * 2;
  // A fragments of K step ks: 8 channels of one tap per lane, one M tile each
  auto a_load = [&](int off, uint4 (&dst)[MT]) {
    const char* p = sb + off;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      dst[mt] = *reinterpret_cast<const uint4*>(p + ((mt >> 2) * QHY + (mt & 3)) * QHZ * kC * 2);
  };
  // software pipeline: the next step's A fragments (LDS) and B fragments
  // (global; uniform base + lane offset) are requested before this step's
  // matrix products are issued; chunk offsets are read two steps ahead
  uint4 A0[MT], A1[MT];
  a_load(s_off[kb], A0);
  int off_next = s_off[4 + kb];
  // the weight fragments are the same for every tile: an opaque copy of the
  // pointer per tile keeps them from being hoisted out of the tile loop
  // (all 42 would then stay live in registers)
  const uint4* wp = wpk;
  asm volatile("" : "+s"(wp));
  uint4 nb0 = wp[l], nb1 = (wp + 64)[l];
#pragma unroll
  for (int ks = 0; ks < kKSteps; ++ks) {
    uint4(&cur)[MT] = (ks & 1) ? A1 : A0;
    uint4(&nxt)[MT] = (ks & 1) ? A0 : A1;
    const bf16x8 b0 = __builtin_bit_cast(bf16x8, nb0);
    const bf16x8 b1 = __builtin_bit_cast(bf16x8, nb1);
    if (ks + 1 < kKSteps) {
      nb0 = (wp + ((ks + 1) * 2 + 0) * 64)[l];
      nb1 = (wp + ((ks + 1) * 2 + 1) * 64)[l];
      a_load(off_next, nxt);
      if (ks + 2 < kKSteps) off_next = s_off[4 * (ks + 2) + kb];
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const bf16x8 a = __builtin_bit_cast(bf16x8, cur[mt]);
      acc[mt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc[mt][0], 0, 0, 0);
      if constexpr (NT == 2) acc[mt][NT - 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc[mt][NT - 1], 0, 0, 0);
    }
  }
  // The next tile's box is loaded now, behind the last weight-fragment load
  // (vector loads retire in order, so a box load issued before the products
  // would hold up the first weight fragment), and lands while the epilogue
  // runs.  The last tile reloads its own box: unconditional loads keep the
  // box in registers.
  u32x4 box[kQBoxPer];
  __builtin_amdgcn_sched_barrier(0);   // keep the box loads behind the products
  qbox_load(in, nx0, ny0, nz0, m, lg, box);
  if constexpr (MODE == 2) {
    // column 0 of D: lane (row 0, kb) holds cells 4 kb .. 4 kb + 3 of each M tile,
    // four consecutive z cells (16-byte aligned in the dense layout)
    if (row == 0) {
      const float bo = bias_reg[0];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        int mx, my, mz;
        qcell(w * MT + mt, 4 * kb, mx, my, mz);
        *reinterpret_cast<float4*>(out1 + didx(x0 + mx, y0 + my, z0 + mz, m, lg)) =
            float4{acc[mt][0][0] + bo, acc[mt][0][1] + bo, acc[mt][0][2] + bo, acc[mt][0][3] + bo};
      }
    }
  } else {
  __syncthreads();
  float* sf = reinterpret_cast<float*>(s);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int o = nt * 16 + row;
      if (o < kC) {
        const float bo = bias_reg[nt];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int mx, my, mz;
          qcell(w * MT + mt, 4 * kb + r, mx, my, mz);
          sf[((mx * QY + my) * QZ + mz) * kC + o] = acc[mt][nt][r] + bo;
        }
      }
    }
  __syncthreads();
  static_assert(kQTile * 3 % 256 == 0, "whole passes of the epilogue");
#pragma unroll
  for (int pass = 0; pass < kQTile * 3 / 256; ++pass) {
    const int q = (int)threadIdx.x + pass * 256;
    const int cell = q / 3, part = q % 3;
    const int mx = cell / (QY * QZ), my = (cell / QZ) % QY, mz = cell % QZ;
    const int64_t g = didx(x0 + mx, y0 + my, z0 + mz, m, lg) * kC + part * 8;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = sf[cell * kC + part * 8 + e];
    if (MODE == 0) {
      float zr[8], ar[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        zr[e] = bfr(v[e]);
        ar[e] = gelu(zr[e]);
      }
      if (out_z) *reinterpret_cast<uint4*>(out_z + g) = pack8(zr);
      *reinterpret_cast<uint4*>(out_a + g) = pack8(ar);
    } else {
      float zp[8], gr[8];
      unpack8(*reinterpret_cast<const uint4*>(zprev + g), zp);
#pragma unroll
      for (int e = 0; e < 8; ++e) gr[e] = v[e] * gelu_grad(zp[e]);
      *reinterpret_cast<uint4*>(out_z + g) = pack8(gr);
    }
  }
  }
  __syncthreads();   // every output has been read back from the buffer
  if (has_next) qbox_store(s, box);
  x0 = nx0;
  y0 = ny0;
  z0 = nz0;
  __syncthreads();   // the next tile's box is complete
  }
}

// ---------------------------------------------------------------------------
// Forward 24 -> 24 convolution marching along x (grids of 32^3 and up).
// A workgroup owns a 16 x 16 (y, z) column segment of kXSeg planes.  Input
// plane x' (its 18 x 18 halo in LDS) meets all three planes of the weights:
// it adds to outputs x' + 1 (taps dx = -1), x' (dx = 0) and x' - 1 (dx = +1),
// whose accumulators stay in registers; output x' - 1 is then complete.  So
// each input cell's 24 channels are read from LDS once per in-plane tap
// (9 times) instead of once per tap (27 times), and the K dimension is
// (dy, dz, channel) in 28 chunks of 8 (7 MFMA steps of 32, one chunk of zero
// weights).  Eight waves, each four 16-cell M tiles (z lines) by one 16-wide
// N tile (output channels 0-15 or 16-23), two waves per SIMD so that one
// wave's epilogue runs beside the other's matrix products; each wave's weight
// fragments are loaded once into registers.  The waves of channels 16-23 pack
// two x-offsets into one 16-column tile (two products per M tile and plane
// instead of three; the partial sums move between the tile's halves by DPP).
// Every output's sum starts from its channel's bias.  A finished output plane
// is staged in LDS and stored to memory during the next step's matrix
// products (not in the barrier-bound gap between steps).  The same products
// per output as k_conv24<0> (bf16 products exact in FP32, FP32 sums in
// another order).
// ---------------------------------------------------------------------------
constexpr int kXY = 16, kXZ = 16;                        // (y, z) tile of a column
constexpr int kXHY = kXY + 2, kXHZ = kXZ + 2;            // halo plane 18 x 18
constexpr int kXHalo = kXHY * kXHZ;                      // 324 cells
constexpr int kXPlaneVec = kXHalo * 3;                   // 16-byte pieces of a halo plane: 972
constexpr int kXThreads = 512, kXMT = 4;                 // eight waves: four M tiles x one N tile each
constexpr int kXPlanePer = (kXPlaneVec + kXThreads - 1) / kXThreads;   // 2 per thread
constexpr int kXTile = kXY * kXZ;                        // 256 output cells per plane
constexpr int kXKSteps = 7;                              // 28 chunks of 8 (9 in-plane taps x 3 + 1 zero)
constexpr int kXPackVecs = 3 * kXKSteps * 2 * 64;        // (dx, step, N tile, lane)
constexpr int kXPairVecs = kXKSteps * 2 * 64;            // paired channels 16-23: (step, tile, lane)
constexpr int kXSegMax = 64;                             // planes per workgroup (fewer on small grids)

// B fragment (dxi, ks, nt) at lane l: W[o][c][tap] for o = 16 nt + (l & 15)
// and chunk j = 4 ks + (l >> 4): in-plane tap j / 3 = 3 (dy + 1) + (dz + 1),
// channels 8 (j % 3) ..; tap = 9 dxi + 3 (dy + 1) + (dz + 1).  Zero for j = 27
// and o >= 24.  After them, the paired fragments of output channels 16-23
// (u, ks) at lane l, column d = l & 15: u = 0 holds o = 16 + d with dxi = 0
// in columns 0-7 and o = 16 + d - 8 with dxi = 1 in columns 8-15; u = 1 holds
// o = 16 + d with dxi = 2 in columns 0-7 and zeros in columns 8-15.
__global__ void k_pack_xmarch(const float* __restrict__ W, uint4* __restrict__ wpk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kXPackVecs + kXPairVecs) return;
  int o, j, dxi;
  const int l = i & 63;
  j = 4 * (((i >= kXPackVecs ? i - kXPackVecs : i) >> 7) % kXKSteps) + (l >> 4);
  if (i < kXPackVecs) {
    o = ((i >> 6) & 1) * 16 + (l & 15);
    dxi = (i >> 7) / kXKSteps;
  } else {
    const int u = ((i - kXPackVecs) >> 6) & 1, d = l & 15;
    o = d < 8 ? 16 + d : (u == 0 ? 8 + d : kC);
    dxi = u == 0 ? (d < 8 ? 0 : 1) : 2;
  }
  bf16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (o < kC && j < 27) {
    const int tap = 9 * dxi + j / 3, cb = (j % 3) * 8;
    for (int e = 0; e < 8; ++e) v[e] = f2bf(W[(o * kC + cb + e) * kTaps + tap]);
  }
  wpk[i] = *reinterpret_cast<const uint4*>(v);
}

__device__ __forceinline__ void xplane_load(const bf16_t* __restrict__ in, int x, int y0, int z0, int m, int lg,
                                            u32x4 (&v)[kXPlanePer]) {
#pragma unroll
  for (int r = 0; r < kXPlanePer; ++r) {
    const int q = min((int)threadIdx.x + r * kXThreads, kXPlaneVec - 1);
    const int cell = q / 3, part = q % 3;
    const int hy = cell / kXHZ, hz = cell % kXHZ;
    v[r] = *reinterpret_cast<const u32x4*>(in + didx(x, y0 - 1 + hy, z0 - 1 + hz, m, lg) * kC + part * 8);
  }
}
__device__ __forceinline__ void xplane_store(bf16_t* sp, const u32x4 (&v)[kXPlanePer]) {
#pragma unroll
  for (int r = 0; r < kXPlanePer; ++r) {
    const int q = threadIdx.x + r * kXThreads;
    if (q < kXPlaneVec) *reinterpret_cast<u32x4*>(sp + q * 8) = v[r];
  }
}

__global__ __launch_bounds__(kXThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_conv24_xmarch(
    int lg, int seg, const bf16_t* __restrict__ in, const uint4* __restrict__ wpk, const float* __restrict__ bias,
    bf16_t* __restrict__ out_z, bf16_t* __restrict__ out_a) {
  __shared__ __attribute__((aligned(16))) bf16_t sp[2][kXHalo * kC];     // halo planes (double buffer)
  __shared__ __attribute__((aligned(16))) bf16_t se[2][kXTile * kC];     // a of a finished plane
  __shared__ __attribute__((aligned(16))) bf16_t sz[2][kXTile * kC];     // z of a finished plane
  const int n = 1 << lg, m = n - 1;
  const int nseg = n / seg, tyz = n / kXY;
  const int bid = (int)xcd_block();
  const int col = bid / nseg, xs = (bid % nseg) * seg;
  const int y0 = (col / tyz) * kXY, z0 = (col % tyz) * kXZ;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, row = l & 15, kb = l >> 4;
  // wave w: output channels 16 nt .. (N tile nt = w / 4) of the z lines y = 4 (w % 4) + mt
  const int nt = __builtin_amdgcn_readfirstlane(w >> 2), y1 = kXMT * (w & 3);
  bf16x8 B[3][kXKSteps];   // this wave's weight fragments, all in registers
  if (nt == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int ks = 0; ks < kXKSteps; ++ks) B[d][ks] = __builtin_bit_cast(bf16x8, wpk[((d * kXKSteps + ks) * 2) * 64 + l]);
  } else {   // the paired fragments of channels 16-23 in B[0] and B[1]
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int ks = 0; ks < kXKSteps; ++ks)
        B[u][ks] = __builtin_bit_cast(bf16x8, wpk[kXPackVecs + (ks * 2 + u) * 64 + l]);
  }
  const int o = nt * 16 + row;   // this lane's output channel
  const float bo = o < kC ? bias[o] : 0.f;
  // A-fragment byte offsets: chunk j = 4 ks + kb shifted by its in-plane tap
  int aoff[kXKSteps];
#pragma unroll
  for (int ks = 0; ks < kXKSteps; ++ks) {
    const int j = min(4 * ks + kb, 26);   // the zero-weight chunk 27 reads chunk 26's inputs
    const int dy = j / 9 - 1, dz = (j / 3) % 3 - 1, cp = j % 3;
    aoff[ks] = (((y1 + 1 + dy) * kXHZ + (row + 1 + dz)) * kC + cp * 8) * 2;
  }
  // four accumulator sets rotate: at step i, set i % 4 completes output
  // xs - 2 + i, sets (i + 1) % 4 and (i + 2) % 4 take the next two, and the
  // epilogue of set (i - 1) % 4 (output xs - 3 + i, completed one step
  // earlier) runs between this step's matrix products.  A set starts from
  // its lane's channel bias.
  f32x4 acc[4][kXMT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int mt = 0; mt < kXMT; ++mt) acc[a][mt] = f32x4{bo, bo, bo, bo};
  {
    u32x4 v[kXPlanePer];
    xplane_load(in, xs - 1, y0, z0, m, lg, v);
    xplane_store(sp[0], v);
  }
  __syncthreads();
  const int steps = seg + 3;   // input planes xs - 1 .. xs + seg, then one step for the last epilogue
  // one output value of the epilogue: M tile mt, row group entry r
  auto epilogue_value = [&](float v, int mt, int r, bf16_t* e_a, bf16_t* e_z) {
    if (o < kC) {
      const int cell = (y1 + mt) * kXZ + 4 * kb + r;
      const float zr = bfr(v);   // (the bias is in the sum)
      e_a[cell * kC + o] = f2bf(gelu(zr));
      if (out_z) e_z[cell * kC + o] = f2bf(zr);
    }
  };
  // global stores of a finished output plane from its LDS buffers
  auto store_plane = [&](int x, const bf16_t* e_a, const bf16_t* e_z) {
#pragma unroll
    for (int r = 0; r < (kXTile * 3 + kXThreads - 1) / kXThreads; ++r) {
      const int q = t + r * kXThreads;
      if (q >= kXTile * 3) break;
      const int cell = q / 3, part = q % 3;
      const int64_t g = didx(x, y0 + cell / kXZ, z0 + cell % kXZ, m, lg) * kC + part * 8;
      *reinterpret_cast<uint4*>(out_a + g) = *reinterpret_cast<const uint4*>(&e_a[q * 8]);
      if (out_z) *reinterpret_cast<uint4*>(out_z + g) = *reinterpret_cast<const uint4*>(&e_z[q * 8]);
    }
  };
  auto step = [&](const int i, auto R_) {
    constexpr int R = decltype(R_)::value;
    constexpr int R1 = (R + 1) % 4, R2 = (R + 2) % 4, RP = (R + 3) % 4;
    const bool has_plane = i < seg + 2;          // input plane xs - 1 + i exists
    const bool has_next = i + 1 < seg + 2;
    const bool prev_ok = i >= 3;                 // output xs - 3 + i lies in the segment
    bf16_t* e_a = se[(i + 1) & 1];
    bf16_t* e_z = sz[(i + 1) & 1];
    u32x4 pf[kXPlanePer];
    if (has_next) xplane_load(in, xs + i, y0, z0, m, lg, pf);
    if (has_plane) {
      const char* base = reinterpret_cast<const char*>(sp[i & 1]);
      u32x4 A0[kXMT], A1[kXMT];
#pragma unroll
      for (int mt = 0; mt < kXMT; ++mt) A0[mt] = *reinterpret_cast<const u32x4*>(base + aoff[0] + mt * kXHZ * kC * 2);
#pragma unroll
      for (int ks = 0; ks < kXKSteps; ++ks) {
        u32x4(&cur)[kXMT] = (ks & 1) ? A1 : A0;
        u32x4(&nxt)[kXMT] = (ks & 1) ? A0 : A1;
        if (ks + 1 < kXKSteps) {
#pragma unroll
          for (int mt = 0; mt < kXMT; ++mt)
            nxt[mt] = *reinterpret_cast<const u32x4*>(base + aoff[ks + 1] + mt * kXHZ * kC * 2);
        }
#pragma unroll
        for (int mt = 0; mt < kXMT; ++mt) {
          const bf16x8 a = __builtin_bit_cast(bf16x8, cur[mt]);
          acc[R2][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B[0][ks], acc[R2][mt], 0, 0, 0);
          acc[R1][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B[1][ks], acc[R1][mt], 0, 0, 0);
          acc[R][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B[2][ks], acc[R][mt], 0, 0, 0);
        }
        // the output finished two steps ago (in se[i & 1] since the last barrier) goes out
        if (ks == 1 && i >= 4) store_plane(xs - 4 + i, se[i & 1], sz[i & 1]);
        // the previous output's 16 values per lane, spread over the 7 steps
        if (prev_ok) {
#pragma unroll
          for (int v = 0; v < 4 * kXMT; ++v)
            if ((v * kXKSteps) / (4 * kXMT) == ks) epilogue_value(acc[RP][v >> 2][v & 3], v >> 2, v & 3, e_a, e_z);
        }
      }
    } else {
      if (i >= 4) store_plane(xs - 4 + i, se[i & 1], sz[i & 1]);
      if (prev_ok) {
#pragma unroll
        for (int v = 0; v < 4 * kXMT; ++v) epilogue_value(acc[RP][v >> 2][v & 3], v >> 2, v & 3, e_a, e_z);
      }
    }
#pragma unroll
    for (int mt = 0; mt < kXMT; ++mt) acc[RP][mt] = f32x4{bo, bo, bo, bo};
    if (has_next) xplane_store(sp[(i + 1) & 1], pf);
    __syncthreads();
  };
  // channels 16-23 (nt = 1): the two x-offsets -1 and 0 share one 16-column
  // product (acc[0], T: output x + 1 in columns 0-7, output x in 8-15) and
  // offset +1 takes columns 0-7 of a second (acc[1], U: output x - 1), so a
  // plane costs two products per M tile instead of three.  After the plane,
  // U's finished output goes to acc[2] for the next step's epilogue, T's
  // columns 8-15 move to U's columns 0-7 and T's columns 0-7 to its 8-15
  // (DPP row rotate / shift by 8, the bias into columns 0-7).
  auto step_pair = [&](const int i) {
    const bool has_plane = i < seg + 2;
    const bool has_next = i + 1 < seg + 2;
    const bool prev_ok = i >= 3;
    bf16_t* e_a = se[(i + 1) & 1];
    bf16_t* e_z = sz[(i + 1) & 1];
    u32x4 pf[kXPlanePer];
    if (has_next) xplane_load(in, xs + i, y0, z0, m, lg, pf);
    if (has_plane) {
      const char* base = reinterpret_cast<const char*>(sp[i & 1]);
      u32x4 A0[kXMT], A1[kXMT];
#pragma unroll
      for (int mt = 0; mt < kXMT; ++mt) A0[mt] = *reinterpret_cast<const u32x4*>(base + aoff[0] + mt * kXHZ * kC * 2);
#pragma unroll
      for (int ks = 0; ks < kXKSteps; ++ks) {
        u32x4(&cur)[kXMT] = (ks & 1) ? A1 : A0;
        u32x4(&nxt)[kXMT] = (ks & 1) ? A0 : A1;
        if (ks + 1 < kXKSteps) {
#pragma unroll
          for (int mt = 0; mt < kXMT; ++mt)
            nxt[mt] = *reinterpret_cast<const u32x4*>(base + aoff[ks + 1] + mt * kXHZ * kC * 2);
        }
#pragma unroll
        for (int mt = 0; mt < kXMT; ++mt) {
          const bf16x8 a = __builtin_bit_cast(bf16x8, cur[mt]);
          acc[0][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B[0][ks], acc[0][mt], 0, 0, 0);
          acc[1][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B[1][ks], acc[1][mt], 0, 0, 0);
        }
        if (ks == 1 && i >= 4) store_plane(xs - 4 + i, se[i & 1], sz[i & 1]);
        if (prev_ok) {
#pragma unroll
          for (int v = 0; v < 4 * kXMT; ++v)
            if ((v * kXKSteps) / (4 * kXMT) == ks) epilogue_value(acc[2][v >> 2][v & 3], v >> 2, v & 3, e_a, e_z);
        }
      }
#pragma unroll
      for (int mt = 0; mt < kXMT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc[2][mt][r] = acc[1][mt][r];
          // (the element goes through a named scalar: a bit cast of the
          // element expression itself compiled to element 0)
          const float tvf = acc[0][mt][r];
          const int rot = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, tvf), 0x128, 0xF, 0xF, false);
          // (columns 0-7 have no source lane: they keep `old`, the channel bias)
          const int shr = __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, bo), __builtin_bit_cast(int, tvf), 0x118,
                                                      0xF, 0xF, false);
          acc[1][mt][r] = __builtin_bit_cast(float, rot);
          acc[0][mt][r] = __builtin_bit_cast(float, shr);
        }
    } else {
      if (i >= 4) store_plane(xs - 4 + i, se[i & 1], sz[i & 1]);
      if (prev_ok) {
#pragma unroll
        for (int v = 0; v < 4 * kXMT; ++v) epilogue_value(acc[2][v >> 2][v & 3], v >> 2, v & 3, e_a, e_z);
      }
    }
    if (has_next) xplane_store(sp[(i + 1) & 1], pf);
    __syncthreads();
  };
  if (nt == 0) {
    for (int i = 0; i < steps; i += 4) {
      step(i, std::integral_constant<int, 0>{});
      if (i + 1 < steps) step(i + 1, std::integral_constant<int, 1>{});
      if (i + 2 < steps) step(i + 2, std::integral_constant<int, 2>{});
      if (i + 3 < steps) step(i + 3, std::integral_constant<int, 3>{});
    }
  } else {
    for (int i = 0; i < steps; ++i) step_pair(i);
  }
  store_plane(xs + seg - 1, se[steps & 1], sz[steps & 1]);   // the last output (its barrier was the last step's)
}

// ---------------------------------------------------------------------------
// Forward 24 -> 1 (last) layer marching along x on the matrix cores (grids
// of 32^3 and up): the column segments and halo planes of k_conv24_xmarch,
// four waves of four z lines each.  The three x-planes of the weights are
// the N dimension of the products (columns 0, 1, 2; the rest zero), so one
// 16x16x32 product per K step takes an input plane's contributions to the
// three output planes it touches: column d (lane d of each 16-lane row) goes
// to output x + 1 - d.  Each lane keeps one running sum that moves one lane
// up per input plane (a DPP row shift, zero into lane 0) before the plane's
// column is added, so lane d holds output x + 1 - d and lane 2 a finished
// one.
// ---------------------------------------------------------------------------
constexpr int kO1Threads = 256;
constexpr int kO1PlanePer = (kXPlaneVec + kO1Threads - 1) / kO1Threads;   // 4 pieces per thread
constexpr int kO1PackVecs = kXKSteps * 64;

// fragment ks at lane l: W[0][cb + e][tap] for column d = l & 15 < 3, chunk
// j = 4 ks + (l >> 4) < 27 (tap 9 d + j / 3, channels cb = 8 (j % 3) ...)
__global__ void k_pack_out1_mfma(const float* __restrict__ W, uint4* __restrict__ wpk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kO1PackVecs) return;
  const int l = i & 63, ks = i >> 6;
  const int d = l & 15, j = 4 * ks + (l >> 4);
  bf16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (d < 3 && j < 27) {
    const int tap = 9 * d + j / 3, cb = (j % 3) * 8;
    for (int e = 0; e < 8; ++e) v[e] = f2bf(W[(cb + e) * kTaps + tap]);
  }
  wpk[i] = *reinterpret_cast<const uint4*>(v);
}

__global__ __launch_bounds__(kO1Threads) __attribute__((amdgpu_waves_per_eu(4))) void k_conv_out1_mfma(int lg, int seg, const bf16_t* __restrict__ in,
                                                              const uint4* __restrict__ wpk,
                                                              const float* __restrict__ bias,
                                                              float* __restrict__ out1) {
  __shared__ __attribute__((aligned(16))) bf16_t sp[2][kXHalo * kC];   // halo planes (double buffer)
  const int n = 1 << lg, m = n - 1;
  const int nseg = n / seg, tyz = n / kXY;
  const int bid = (int)xcd_block();
  const int col = bid / nseg, xs = (bid % nseg) * seg;
  const int y0 = (col / tyz) * kXY, z0 = (col % tyz) * kXZ;
  const int t = threadIdx.x, w = t >> 6, l = t & 63, row = l & 15, kb = l >> 4;
  const int y1 = kXMT * w;   // this wave's z lines y1 .. y1 + 3
  bf16x8 B[kXKSteps];
#pragma unroll
  for (int ks = 0; ks < kXKSteps; ++ks) B[ks] = __builtin_bit_cast(bf16x8, wpk[ks * 64 + l]);
  const float b0 = bias[0];
  int aoff[kXKSteps];
#pragma unroll
  for (int ks = 0; ks < kXKSteps; ++ks) {
    const int j = min(4 * ks + kb, 26);   // the zero-weight chunk 27 reads chunk 26's inputs
    const int dy = j / 9 - 1, dz = (j / 3) % 3 - 1, cp = j % 3;
    aoff[ks] = (((y1 + 1 + dy) * kXHZ + (row + 1 + dz)) * kC + cp * 8) * 2;
  }
  auto load = [&](int x, u32x4 (&v)[kO1PlanePer]) {
#pragma unroll
    for (int r = 0; r < kO1PlanePer; ++r) {
      const int q = min(t + r * kO1Threads, kXPlaneVec - 1);
      const int cell = q / 3, part = q % 3;
      v[r] = *reinterpret_cast<const u32x4*>(in + didx(x, y0 - 1 + cell / kXHZ, z0 - 1 + cell % kXHZ, m, lg) * kC +
                                             part * 8);
    }
  };
  auto store = [&](bf16_t* dst, const u32x4 (&v)[kO1PlanePer]) {
#pragma unroll
    for (int r = 0; r < kO1PlanePer; ++r) {
      const int q = t + r * kO1Threads;
      if (q < kXPlaneVec) *reinterpret_cast<u32x4*>(dst + q * 8) = v[r];
    }
  };
  f32x4 acc[kXMT];   // lane d of a row: output x + 1 - d after input plane x
#pragma unroll
  for (int mt = 0; mt < kXMT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
  {
    u32x4 v[kO1PlanePer];
    load(xs - 1, v);
    store(sp[0], v);
  }
  __syncthreads();
  const int steps = seg + 2;   // input planes xs - 1 .. xs + seg
  auto step = [&](const int i) {
    const bool has_next = i + 1 < steps;
    u32x4 pf[kO1PlanePer];
    if (has_next) load(xs + i, pf);
    const char* base = reinterpret_cast<const char*>(sp[i & 1]);
    f32x4 c[kXMT];
#pragma unroll
    for (int mt = 0; mt < kXMT; ++mt) c[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kXKSteps; ++ks) {
#pragma unroll
      for (int mt = 0; mt < kXMT; ++mt) {
        const u32x4 av = *reinterpret_cast<const u32x4*>(base + aoff[ks] + mt * kXHZ * kC * 2);
        c[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), B[ks], c[mt], 0, 0, 0);
      }
    }
    // the running sums move one lane up (lane 0 starts a new output), then
    // take this plane's column
#pragma unroll
    for (int mt = 0; mt < kXMT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // (the element goes through a named scalar: a bit cast of the
        // element expression itself compiled to element 0)
        const float cur = acc[mt][r];
        const int up = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, cur), 0x111, 0xF, 0xF, true);
        acc[mt][r] = __builtin_bit_cast(float, up) + c[mt][r];
      }
    if (has_next) store(sp[(i + 1) & 1], pf);
    if (i >= 2 && row == 2) {   // output xs - 2 + i is complete in lane 2 of each row
      const int x = xs - 2 + i;
#pragma unroll
      for (int mt = 0; mt < kXMT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) out1[didx(x, y0 + y1 + mt, z0 + 4 * kb + r, m, lg)] = acc[mt][r] + b0;
    }
    __syncthreads();
  };
  for (int i = 0; i < steps; ++i) step(i);
}

void conv_out1_mfma_launch(int lg, const bf16_t* in, const uint4* wpk, const float* bias, float* out1,
                           hipStream_t s) {
  const int n = 1 << lg;
  const int seg = std::min(kXSegMax, n);
  const int blocks = (n / kXY) * (n / kXZ) * (n / seg);
  hipLaunchKernelGGL(k_conv_out1_mfma, dim3((unsigned)blocks), dim3(kO1Threads), 0, s, lg, seg, in, wpk, bias, out1);
}

void conv24_xmarch_launch(int lg, const bf16_t* in, const uint4* wpk, const float* bias, bf16_t* out_z,
                          bf16_t* out_a, hipStream_t s) {
  const int n = 1 << lg;
  const int seg = std::min(kXSegMax, n);
  const int blocks = (n / kXY) * (n / kXZ) * (n / seg);
  hipLaunchKernelGGL(k_conv24_xmarch, dim3((unsigned)blocks), dim3(kXThreads), 0, s, lg, seg, in, wpk, bias, out_z,
                     out_a);
}

// Launch of the persistent convolution: as many workgroups as the device
// holds at once, at most one per tile.
template <int MODE>
void conv24_launch(int lg, const bf16_t* in, const uint4* wpk, const float* bias, const bf16_t* zprev,
                   bf16_t* out_z, bf16_t* out_a, float* out1, hipStream_t s) {
  static int cap = 0;
  if (cap == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    MG_HIP(hipGetDevice(&dev));
    MG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_conv24<MODE>, 256, 0));
    cap = std::max(1, cus * per_cu);
  }
  const int n = 1 << lg;
  const int n_tiles = (n / QX) * (n / QY) * (n / QZ);
  hipLaunchKernelGGL((k_conv24<MODE>), dim3((unsigned)std::min(n_tiles, cap)), dim3(256), 0, s, lg, n_tiles, in,
                     wpk, bias, zprev, out_z, out_a, out1);
}

// First layer (1 -> 24 + GELU, forward) on the matrix cores: per cell the
// 27 taps of the one input channel are the K dimension (padded to 32); the
// weights are the product's rows (24 outputs in two 16-row tiles) and 16
// cells its columns, so each lane ends with four consecutive channels of one
// cell and stores them to LDS as one 8-byte word.  8 x 8 x 8 cell tiles.  The
// input is the BF16 copy of the network input and the weights are rounded to
// BF16 as in every layer, so the products are exact in FP32 and only the
// summation order is the matrix core's.  The weight fragments come packed
// (k_pack_in1).
// fragment nt at lane (row, kb): W[o][t] for o = 16 nt + row, taps
// t = 8 kb .. 8 kb + 7 (zero beyond the 27 taps and the 24 outputs)
__global__ void k_pack_in1(const float* __restrict__ W, uint4* __restrict__ wpk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * 64) return;
  const int l = i & 63, nt = i >> 6, o = nt * 16 + (l & 15), kb = l >> 4;
  bf16_t v[8];
  for (int j = 0; j < 8; ++j) {
    const int t = 8 * kb + j;
    v[j] = (o < kC && t < kTaps) ? f2bf(W[o * kTaps + t]) : (bf16_t)0;
  }
  wpk[i] = *reinterpret_cast<const uint4*>(v);
}
__global__ __launch_bounds__(256) void k_conv_in1_mfma(int lg, const bf16_t* __restrict__ in,
                                                       const uint4* __restrict__ wpk, const float* __restrict__ bias,
                                                       bf16_t* __restrict__ out_z, bf16_t* __restrict__ out_a) {
  __shared__ bf16_t sx[kQHalo];
  __shared__ __attribute__((aligned(16))) bf16_t sf[kQTile * kC];   // z of the tile, rounded
  const int m = (1 << lg) - 1;
  int x0, y0, z0;
  qtile_origin(lg, (int)xcd_block(), x0, y0, z0);
  {
    // halo cell q = (hx QHY + hy) QHZ + hz, advanced by 256 = 2 QHY QHZ + 5 QHZ + 6
    // per pass; all four loads are issued before the first LDS write
    static_assert(QHY == 10 && QHZ == 10 && kQHalo <= 4 * 256, "the digit steps below");
    const int q0 = threadIdx.x;
    int hx = q0 / 100, hy = (q0 / 10) % 10, hz = q0 % 10;
    bf16_t hv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      hv[k] = in[didx(x0 - 1 + hx, y0 - 1 + hy, z0 - 1 + hz, m, lg)];   // (wrapped: in bounds past the halo too)
      hz += 6;
      hy += 5;
      hx += 2;
      if (hz >= 10) {
        hz -= 10;
        ++hy;
      }
      if (hy >= 10) {
        hy -= 10;
        ++hx;
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (q0 + 256 * k < kQHalo) sx[q0 + 256 * k] = hv[k];
  }
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row = l & 15, kb = l >> 4;
  bf16x8 b[2];
  float bo[2][4];   // biases of this lane's output channels 16 nt + 4 kb + r
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    b[nt] = __builtin_bit_cast(bf16x8, wpk[nt * 64 + l]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = nt * 16 + 4 * kb + r;
      bo[nt][r] = o < kC ? bias[o] : 0.f;
    }
  }
  // this lane's taps 8 kb + j as offsets in the halo box (compile-time per kb;
  // taps past the 27th read tap 26, their weights are zero)
  int toff[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    auto off = [](int t) {
      t = t < kTaps ? t : kTaps - 1;
      return ((t / 9 - 1) * QHY + (t / 3) % 3 - 1) * QHZ + t % 3 - 1;
    };
    toff[j] = kb == 0 ? off(j) : kb == 1 ? off(8 + j) : kb == 2 ? off(16 + j) : off(24 + j);
  }
  __syncthreads();
  constexpr int MT = kQTile / 16 / 4;   // 8 M tiles per wave
  // this lane's cell in M tile 0; M tile mt adds (mt / 4, mt % 4) to its (x, y)
  int mx0, my0, mz0;
  qcell(wv * MT, row, mx0, my0, mz0);
  static_assert(MT == 8, "two x rows of four y lines per wave");
  int tb[8];   // halo index of tap j of the lane's cell in M tile 0
#pragma unroll
  for (int j = 0; j < 8; ++j) tb[j] = ((mx0 + 1) * QHY + (my0 + 1)) * QHZ + (mz0 + 1) + toff[j];
  const int cell0 = (mx0 * QY + my0) * QZ + mz0;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int dh = ((mt >> 2) * QHY + (mt & 3)) * QHZ, dc = ((mt >> 2) * QY + (mt & 3)) * QZ;
    uint16_t ha[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) ha[j] = sx[tb[j] + dh];   // (finite inputs: taps past 26 meet zero weights)
    const bf16x8 a = __builtin_bit_cast(bf16x8, ha);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      // rows: output channels 16 nt + 4 kb + r; column: this lane's cell; the
      // product starts from the channels' biases
      const f32x4 c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          b[nt], a, f32x4{bo[nt][0], bo[nt][1], bo[nt][2], bo[nt][3]}, 0, 0, 0);
      if (nt == 0 || kb < 2) {   // channels 24-31 are padding
        uint2 pk;
        pk.x = pack2(c[0], c[1]);
        pk.y = pack2(c[2], c[3]);
        *reinterpret_cast<uint2*>(sf + (cell0 + dc) * kC + nt * 16 + 4 * kb) = pk;
      }
    }
  }
  __syncthreads();
  // 16-byte piece q of the tile: z run rr = q / 24 (x, y of the tile), piece
  // w = q % 24 of the run's 8 cells x 3 pieces, contiguous in both layouts
  // (the tile lies inside the grid, so no wrap)
  int rr = (int)threadIdx.x / 24, w = (int)threadIdx.x - 24 * rr;
#pragma unroll
  for (int pass = 0; pass < kQTile * 3 / 256; ++pass) {
    const int q = (int)threadIdx.x + pass * 256;
    const int64_t run = ((int64_t)(x0 + (rr >> 3)) << (2 * lg)) + ((int64_t)(y0 + (rr & 7)) << lg) + z0;
    const int64_t g = (run * 3 + w) * 8;
    rr += 10;   // q + 256 = 24 (rr + 10) + w + 16
    w += 16;
    if (w >= 24) {
      w -= 24;
      ++rr;
    }
    const uint4 zv = *reinterpret_cast<const uint4*>(sf + q * 8);
    float zr[8], ar[8];
    unpack8(zv, zr);
#pragma unroll
    for (int e = 0; e < 8; ++e) ar[e] = gelu(zr[e]);
    if (out_z) *reinterpret_cast<uint4*>(out_z + g) = zv;
    *reinterpret_cast<uint4*>(out_a + g) = pack8(ar);
  }
}

// B fragments of a 24 -> nout layer for k_conv24 (nout = 24 or 1): fragment
// (ks, nt) at lane l holds W[o][c][tap] for o = 16 nt + (l & 15) < nout (zero
// otherwise) and the 8 channels of chunk j = 4 ks + (l >> 4) (tap j / 3,
// channels 8 (j % 3) ...), W laid out [nout][24][27].  `transpose_flip` packs
// the input-gradient convolution of a layer W[c][o][tap] ([24][nout][27]):
// W'[o][c][tap] = W[c][o][26 - tap].
__global__ void k_pack24(const float* __restrict__ W, uint4* __restrict__ wpk, int transpose_flip, int nout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kPackVecs) return;
  const int l = i & 63, nt = (i >> 6) & 1, ks = i >> 7;
  const int col = nt * 16 + (l & 15), j = 4 * ks + (l >> 4);
  bf16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (col < nout && j < kChunks) {
    const int tap = j / 3, cb = (j % 3) * 8;
    for (int e = 0; e < 8; ++e) {
      const int c = cb + e;
      const float wv = transpose_flip ? W[(c * nout + col) * kTaps + (kTaps - 1 - tap)] : W[(col * kC + c) * kTaps + tap];
      v[e] = f2bf(wv);
    }
  }
  wpk[i] = *reinterpret_cast<const uint4*>(v);
}

// ---------------------------------------------------------------------------
// input gradient of the last layer (one channel -> 24, vector ALU):
// g = conv(dy, W4 tap-flipped) * gelu'(zprev); w points at the [24][27] block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv_in1_grad(int lg, const float* __restrict__ in, const float* __restrict__ w,
                                                       const bf16_t* __restrict__ zprev, bf16_t* __restrict__ out_g) {
  __shared__ float sx[kHalo];
  __shared__ float sw[kC * kTaps];
  const int m = (1 << lg) - 1;
  int x0, y0, z0;
  tile_origin(lg, blockIdx.x, x0, y0, z0);
  {
    constexpr int kPer = (kHalo + 255) / 256;
    float v[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int q = min((int)threadIdx.x + r * 256, kHalo - 1);
      const int hx = q / (HY * HZ), hy = (q / HZ) % HY, hz = q % HZ;
      v[r] = in[didx(x0 - 1 + hx, y0 - 1 + hy, z0 - 1 + hz, m, lg)];
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r)
      if ((int)threadIdx.x + r * 256 < kHalo) sx[threadIdx.x + r * 256] = v[r];
  }
  for (int q = threadIdx.x; q < kC * kTaps; q += blockDim.x) {
    const int o = q / kTaps, t = q % kTaps;
    sw[q] = bfr(w[o * kTaps + kTaps - 1 - t]);
  }
  __syncthreads();
  int mx, my, mz;
  tile_cell(threadIdx.x, mx, my, mz);
  float v27[kTaps];
#pragma unroll
  for (int t = 0; t < kTaps; ++t) {
    int dx, dy, dz;
    tap_offset(t, dx, dy, dz);
    v27[t] = sx[halo_cell(mx + 1 + dx, my + 1 + dy, mz + 1 + dz)];
  }
  const int64_t g = didx(x0 + mx, y0 + my, z0 + mz, m, lg) * kC;
#pragma unroll 1
  for (int grp = 0; grp < 3; ++grp) {
    float acc[8] = {};
#pragma unroll
    for (int t = 0; t < kTaps; ++t)
#pragma unroll
      for (int o = 0; o < 8; ++o) acc[o] += sw[(grp * 8 + o) * kTaps + t] * v27[t];
    float zp[8], gr[8];
    unpack8(reinterpret_cast<const uint4*>(zprev + g)[grp], zp);
#pragma unroll
    for (int o = 0; o < 8; ++o) gr[o] = acc[o] * gelu_grad(zp[o]);
    reinterpret_cast<uint4*>(out_g + g)[grp] = pack8(gr);
  }
}

// ---------------------------------------------------------------------------
// weight gradients: out[m][n][tap] = sum_p U[p][m] V[p + tap][n] (matrix cores)
// U: [p][24] bf16, V: [p][CV] bf16 (CV = 24 or 1).  Tiles of 2 x 8 x 8 cells;
// MFMA K = 32 cells = four runs of 8 cells along z.  Persistent workgroups;
// wave w owns the taps t = w, w + 4, ...; each writes its partial sums.
// ---------------------------------------------------------------------------
constexpr int CX = 2;                                  // correlation tile: 2 x 8 x 8 cells
constexpr int kCorrCells = CX * TY * TZ;               // 128
constexpr int kRuns = CX * TY;                         // runs of 8 cells along z
constexpr int kCorrKSteps = kCorrCells / 32;           // 4
constexpr int kVX = CX + 2, kVY = TY + 2;              // V box in x, y (z: 8 per shifted copy)
constexpr int kMaxTapsPerWave = (kTaps + 3) / 4;       // 7

template <int CV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_corr(int lg, const bf16_t* __restrict__ U, const bf16_t* __restrict__ V,
                                              float* __restrict__ partials) {
  constexpr int NT = CV > 16 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) bf16_t sU[kC * kCorrCells];            // [m][cell]
  __shared__ __attribute__((aligned(16))) bf16_t sV[3 * CV * kVX * kVY * 8];     // [dz+1][n][vx][vy][z]
  const int n = 1 << lg, m = n - 1;
  const int tnz = n / TZ, tny = n / TY, tnx = n / CX;
  const int tiles = tnx * tny * tnz;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row = l & 15, kb = l >> 4;
  f32x4 acc[kMaxTapsPerWave][2][NT];
#pragma unroll
  for (int ti = 0; ti < kMaxTapsPerWave; ++ti)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[ti][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int z0 = (tile % tnz) * TZ, y0 = ((tile / tnz) % tny) * TY, x0 = (tile / (tnz * tny)) * CX;
    __syncthreads();
    // U transposed: sU[m][cell]; V with halo, three copies shifted by
    // dz = -1, 0, +1.  All loads are issued before the first LDS store.
    constexpr int kUVec = kCorrCells * 3, kUPer = (kUVec + 255) / 256;
    constexpr int kVItems = 3 * kVX * kVY * 8, kVPer = (kVItems + 255) / 256;
    uint4 ru[kUPer];
#pragma unroll
    for (int r = 0; r < kUPer; ++r) {
      const int q = min((int)threadIdx.x + r * 256, kUVec - 1);
      const int cell = q / 3, part = q % 3;
      const int cx = cell / (TY * TZ), cy = (cell / TZ) % TY, cz = cell % TZ;
      ru[r] = *reinterpret_cast<const uint4*>(U + didx(x0 + cx, y0 + cy, z0 + cz, m, lg) * kC + part * 8);
    }
#pragma unroll
    for (int r = 0; r < kUPer; ++r) {
      const int q = threadIdx.x + r * 256;
      if (q < kUVec) {
        const int cell = q / 3, part = q % 3;
        const bf16_t* pv = reinterpret_cast<const bf16_t*>(&ru[r]);
#pragma unroll
        for (int e = 0; e < 8; ++e) sU[(part * 8 + e) * kCorrCells + cell] = pv[e];
      }
    }
    // V: all items at once for one channel; one item (three loads) at a time
    // for 24 channels, which keeps the kernel at two waves per SIMD
    using VLoad = typename std::conditional<CV == 1, bf16_t, uint4>::type;
    constexpr int kBatch = CV == 1 ? kVPer : 1;
#pragma unroll 1
    for (int r0 = 0; r0 < kVPer; r0 += kBatch) {
      VLoad rv[kBatch][CV == 1 ? 1 : 3];
#pragma unroll
      for (int r = 0; r < kBatch; ++r) {
        const int q = min((int)threadIdx.x + (r0 + r) * 256, kVItems - 1);
        const int z = q % 8, vy = (q / 8) % kVY, vx = (q / (8 * kVY)) % kVX, sh = q / (8 * kVY * kVX);
        const int64_t g = didx(x0 - 1 + vx, y0 - 1 + vy, z0 + z + sh - 1, m, lg);
        if constexpr (CV == 1) {
          rv[r][0] = V[g];
        } else {
#pragma unroll
          for (int k = 0; k < 3; ++k) rv[r][k] = reinterpret_cast<const uint4*>(V + g * kC)[k];
        }
      }
#pragma unroll
      for (int r = 0; r < kBatch; ++r) {
        const int q = threadIdx.x + (r0 + r) * 256;
        if (r0 + r < kVPer && q < kVItems) {
          const int z = q % 8, vy = (q / 8) % kVY, vx = (q / (8 * kVY)) % kVX, sh = q / (8 * kVY * kVX);
          if constexpr (CV == 1) {
            sV[((sh * kVX + vx) * kVY + vy) * 8 + z] = rv[r][0];
          } else {
            const bf16_t* vv = reinterpret_cast<const bf16_t*>(&rv[r][0]);
#pragma unroll
            for (int c = 0; c < kC; ++c) sV[(((sh * CV + c) * kVX + vx) * kVY + vy) * 8 + z] = vv[c];
          }
        }
      }
    }
    __syncthreads();
    for (int ks = 0; ks < kCorrKSteps; ++ks) {
      const int run = ks * 4 + kb;                  // this lane's run of 8 cells
      const int rx = run / TY, ry = run % TY;
      bf16x8 a[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const int mm = mt * 16 + row;
        uint4 raw = {0u, 0u, 0u, 0u};
        if (mm < kC) raw = *reinterpret_cast<const uint4*>(sU + mm * kCorrCells + run * 8);
        a[mt] = __builtin_bit_cast(bf16x8, raw);
      }
#pragma unroll
      for (int ti = 0; ti < kMaxTapsPerWave; ++ti) {
        const int t = w + 4 * ti;
        if (t >= kTaps) break;
        int dx, dy, dz;
        tap_offset(t, dx, dy, dz);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int nn = nt * 16 + row;
          uint4 raw = {0u, 0u, 0u, 0u};
          if (nn < CV)
            raw = *reinterpret_cast<const uint4*>(sV + ((((dz + 1) * CV + nn) * kVX + rx + 1 + dx) * kVY + ry + 1 + dy) * 8);
          const bf16x8 b = __builtin_bit_cast(bf16x8, raw);
#pragma unroll
          for (int mt = 0; mt < 2; ++mt)
            acc[ti][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, acc[ti][mt][nt], 0, 0, 0);
        }
      }
    }
  }
  float* out = partials + (int64_t)blockIdx.x * (kC * CV * kTaps);
#pragma unroll
  for (int ti = 0; ti < kMaxTapsPerWave; ++ti) {
    const int t = w + 4 * ti;
    if (t >= kTaps) break;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int nn = nt * 16 + row;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int mm = mt * 16 + 4 * kb + r;
          if (mm < kC && nn < CV) out[(mm * CV + nn) * kTaps + t] = acc[ti][mt][nt][r];
        }
      }
  }
}

// grad[i'] += sum over workgroups of partials[w][i], i' = i or its tap-flipped index
__global__ void k_reduce_partials(const float* __restrict__ partials, int nwg, int size, int flip,
                                  float* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= size) return;
  double s = 0.0;
  for (int w = 0; w < nwg; ++w) s += (double)partials[(int64_t)w * size + i];
  const int t = i % kTaps;
  grad[flip ? (i - t + (kTaps - 1 - t)) : i] += (float)s;
}

// per-workgroup sums of each of 24 channels of a [p][24] bf16 field (bias gradients)
__global__ __launch_bounds__(256) void k_colsum24(int64_t np, const bf16_t* __restrict__ g, float* __restrict__ partials) {
  __shared__ float red[256];
  const int c = threadIdx.x % kC, lane_group = threadIdx.x / kC;   // 10 groups of 24 (240 threads)
  float acc = 0.f;
  if (threadIdx.x < 240)
    for (int64_t p = (int64_t)blockIdx.x * 10 + lane_group; p < np; p += (int64_t)gridDim.x * 10) acc += bf2f(g[p * kC + c]);
  red[threadIdx.x] = threadIdx.x < 240 ? acc : 0.f;
  __syncthreads();
  if (threadIdx.x < kC) {
    float s = 0.f;
    for (int k = 0; k < 10; ++k) s += red[k * kC + threadIdx.x];
    partials[blockIdx.x * kC + threadIdx.x] = s;
  }
}

__global__ void k_reduce_bias(const float* __restrict__ partials, int nwg, int width, float* __restrict__ grad_b) {
  const int c = threadIdx.x;
  if (c >= width) return;
  double s = 0.0;
  for (int w = 0; w < nwg; ++w) s += partials[w * width + c];
  grad_b[c] += (float)s;
}

// per-workgroup sums of an f32 field (bias gradient of the last layer)
__global__ __launch_bounds__(256) void k_sum_f32(int64_t np, const float* __restrict__ x, float* __restrict__ partials) {
  __shared__ float red[256];
  float acc = 0.f;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) acc += x[p];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void k_f32_to_bf16(int64_t np, const float* __restrict__ x, bf16_t* __restrict__ out, float* __restrict__ xr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const bf16_t b = f2bf(x[p]);
  out[p] = b;
  if (xr) xr[p] = bf2f(b);
}

// network input from an oct-major f64 source term: x = bf16(f / rms(f)) (dense)
__global__ void k_input(int lg, const double* __restrict__ f, const double* __restrict__ sc, bf16_t* __restrict__ xb,
                        float* __restrict__ xf) {
  const int64_t n = 1 << lg;
  const int64_t np = n * n * n;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const double ms = sc[1] / (double)np;                  // mean of f^2
  const double inv_rms = ms > 0.0 ? 1.0 / sqrt(ms) : 0.0;
  const int x = (int)(p >> (2 * lg)), y = (int)((p >> lg) & (n - 1)), z = (int)(p & (n - 1));
  const int lno = lg - 1;
  const int64_t o = ((((int64_t)(z >> 1) << lno) + (y >> 1)) << lno) + (x >> 1);
  const bf16_t b = f2bf((float)(f[o * 8 + (x & 1) + 2 * (y & 1) + 4 * (z & 1)] * inv_rms));
  xb[p] = b;
  xf[p] = bf2f(b);
}

// phi0 (oct-major f64) = s * y (dense f32), s = h^2 rms(f); mode 1: t = phi / s (dense f32)
__global__ void k_scale_io(int lg, int mode, const double* __restrict__ sc, const float* __restrict__ y,
                           double* __restrict__ phi0, const double* __restrict__ phi, float* __restrict__ t) {
  const int64_t n = 1 << lg;
  const int64_t np = n * n * n;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const double h = 1.0 / (double)n;
  const double s = h * h * sqrt(sc[1] / (double)np);
  const int x = (int)(p >> (2 * lg)), yy = (int)((p >> lg) & (n - 1)), z = (int)(p & (n - 1));
  const int lno = lg - 1;
  const int64_t o = ((((int64_t)(z >> 1) << lno) + (yy >> 1)) << lno) + (x >> 1);
  const int64_t i = o * 8 + (x & 1) + 2 * (yy & 1) + 4 * (z & 1);
  if (mode == 0) phi0[i] = s * (double)y[p];
  else t[p] = s > 0.0 ? (float)(phi[i] / s) : 0.f;
}

// dL/dy (dense f32) = s * dL/dphi0 (oct-major f32), s = h^2 rms(f) of the last
// field forward: the chain rule through phi0 = s y, s held fixed
__global__ void k_dphi_to_dy(int lg, const double* __restrict__ sc, const float* __restrict__ dphi,
                             float* __restrict__ dy) {
  const int64_t n = 1 << lg;
  const int64_t np = n * n * n;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const double h = 1.0 / (double)n;
  const double s = h * h * sqrt(sc[1] / (double)np);
  const int x = (int)(p >> (2 * lg)), yy = (int)((p >> lg) & (n - 1)), z = (int)(p & (n - 1));
  const int lno = lg - 1;
  const int64_t o = ((((int64_t)(z >> 1) << lno) + (yy >> 1)) << lno) + (x >> 1);
  dy[p] = (float)(s * (double)dphi[o * 8 + (x & 1) + 2 * (yy & 1) + 4 * (z & 1)]);
}

// The same three transforms for n >= 32, staged through LDS so that both
// layouts move in contiguous runs: a tile is 16 x 16 octs (x, z) of one oct
// row in y, i.e. 32 x 2 x 32 cells; its oct side is 16 runs of 128
// consecutive values (16 octs of 8 cells), its dense side 64 runs of 32 z
// cells.  dir 0: rho (oct) -> xb, xf: f = c (rho - mean) (the mean in sc[0])
// scaled to unit rms, dense, BF16 values; dir 1: y (dense) -> phi0 = s y (oct);
// dir 2: phi (oct) -> t = phi / s (dense).
constexpr int kIoT = 32;
__global__ __launch_bounds__(256) void k_io_tiled(int lg, int dir, const double* __restrict__ sc, double c,
                                                  const double* __restrict__ oin, const float* __restrict__ din,
                                                  double* __restrict__ oout, float* __restrict__ dout,
                                                  bf16_t* __restrict__ dout_b) {
  __shared__ float st[kIoT * 2 * kIoT];   // [x][y][z] of the tile, z fastest
  const int n = 1 << lg, no = n >> 1, tx = n / kIoT;
  const int64_t np = (int64_t)n * n * n;
  const int b = (int)blockIdx.x;
  const int xt = b % tx, yo = (b / tx) % no, zt = b / (tx * no);
  const int x0 = xt * kIoT, y0 = 2 * yo, z0 = zt * kIoT, xo0 = x0 >> 1, zo0 = z0 >> 1;
  const double ms = sc[1] / (double)np;                                 // mean of f^2
  const double inv_rms = ms > 0.0 ? 1.0 / sqrt(ms) : 0.0;
  const double h = 1.0 / (double)n, sf = h * h * sqrt(ms);
  constexpr int kPer = kIoT * 2 * kIoT / 256;                           // 8
  if (dir != 1) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = (int)threadIdx.x + 256 * k, row = e >> 7, w = e & 127, cc = w & 7;
      const double u = oin[(((int64_t)(zo0 + row) * no + yo) * no + xo0 + (w >> 3)) * 8 + cc];
      const int xl = 2 * (w >> 3) + (cc & 1), yl = (cc >> 1) & 1, zl = 2 * row + (cc >> 2);
      if (dir == 0) {
        const double v = c * (u - sc[0]);   // the right-hand side f, as the solver forms it
        st[(xl * 2 + yl) * kIoT + zl] = bfr((float)(v * inv_rms));
      } else {
        st[(xl * 2 + yl) * kIoT + zl] = sf > 0.0 ? (float)(u / sf) : 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int d = (int)threadIdx.x + 256 * k, zl = d & (kIoT - 1), yl = (d >> 5) & 1, xl = d >> 6;
      const int64_t p = ((int64_t)(x0 + xl) * n + y0 + yl) * n + z0 + zl;
      dout[p] = st[d];
      if (dir == 0) dout_b[p] = f2bf(st[d]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int d = (int)threadIdx.x + 256 * k, zl = d & (kIoT - 1), yl = (d >> 5) & 1, xl = d >> 6;
      st[d] = din[((int64_t)(x0 + xl) * n + y0 + yl) * n + z0 + zl];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = (int)threadIdx.x + 256 * k, row = e >> 7, w = e & 127, cc = w & 7;
      const int xl = 2 * (w >> 3) + (cc & 1), yl = (cc >> 1) & 1, zl = 2 * row + (cc >> 2);
      oout[(((int64_t)(zo0 + row) * no + yo) * no + xo0 + (w >> 3)) * 8 + cc] = sf * (double)st[(xl * 2 + yl) * kIoT + zl];
    }
  }
}
inline unsigned io_tiles(int lg) {
  const int n = 1 << lg;
  return (unsigned)((n / kIoT) * (n / kIoT) * (n / 2));
}

// per-workgroup sums of t^2 (f64)
__global__ __launch_bounds__(256) void k_sumsq(int64_t np, const float* __restrict__ t, double* __restrict__ partials) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x)
    acc += (double)t[p] * (double)t[p];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// relative MSE: dy = 2 (y - t) / sum(t^2) and per-workgroup sums of (y - t)^2 / sum(t^2)
__global__ __launch_bounds__(256) void k_mse(int64_t np, const float* __restrict__ y, const float* __restrict__ t,
                                             const double* __restrict__ sum_t2, float* __restrict__ dy,
                                             double* __restrict__ partials) {
  __shared__ double red[256];
  const double st2 = sum_t2[0] > 0.0 ? sum_t2[0] : 1.0;
  const float scale = (float)(2.0 / st2);
  double acc = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    const float r = y[p] - t[p];
    dy[p] = scale * r;
    acc += (double)r * (double)r;
  }
  red[threadIdx.x] = acc / st2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// warm-start residual in lattice units: R = x - (sum of 6 neighbours of y - 6 y); partial sums of R^2
__global__ __launch_bounds__(256) void k_res_r(int lg, const float* __restrict__ x, const float* __restrict__ y,
                                               float* __restrict__ R, double* __restrict__ partials) {
  __shared__ double red[256];
  const int n = 1 << lg, m = n - 1;
  const int64_t np = (int64_t)n * n * n;
  double acc = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    const int px = (int)(p >> (2 * lg)), py = (int)((p >> lg) & m), pz = (int)(p & m);
    const float nb = y[didx(px - 1, py, pz, m, lg)] + y[didx(px + 1, py, pz, m, lg)] + y[didx(px, py - 1, pz, m, lg)] +
                     y[didx(px, py + 1, pz, m, lg)] + y[didx(px, py, pz - 1, m, lg)] + y[didx(px, py, pz + 1, m, lg)];
    const float r = x[p] - (nb - 6.f * y[p]);
    R[p] = r;
    acc += (double)r * (double)r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// dy += -(2 w / N) Lap(R)  (gradient of w mean(R^2); the Laplacian is symmetric)
__global__ void k_res_dy(int lg, const float* __restrict__ R, float w, float* __restrict__ dy) {
  const int n = 1 << lg, m = n - 1;
  const int64_t np = (int64_t)n * n * n;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int px = (int)(p >> (2 * lg)), py = (int)((p >> lg) & m), pz = (int)(p & m);
  const float nb = R[didx(px - 1, py, pz, m, lg)] + R[didx(px + 1, py, pz, m, lg)] + R[didx(px, py - 1, pz, m, lg)] +
                   R[didx(px, py + 1, pz, m, lg)] + R[didx(px, py, pz - 1, m, lg)] + R[didx(px, py, pz + 1, m, lg)];
  dy[p] += -(2.f * w / (float)np) * (nb - 6.f * R[p]);
}

__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ mo,
                       float* __restrict__ ve, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * mo[i] + (1.f - b1) * gi;
  const float vi = b2 * ve[i] + (1.f - b2) * gi * gi;
  mo[i] = mi;
  ve[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace
}  // namespace mg

using namespace mg;

// ---------------------------------------------------------------------------
// the network handle
// ---------------------------------------------------------------------------
struct mgnn_s {
  DevBuf params, grads, adam_m, adam_v;
  int64_t step = 0;
  int n = 0;                                // workspace size (cells per dimension)
  int field_n = 0;                          // n of the last mgnn_forward (0: none since the last raw pass)
  DevBuf xb, xf, y, t, dy, dyb;             // dense [n^3]
  DevBuf Z[4], A[4];                        // [n^3][24] bf16
  DevBuf G[2];                              // gradient ping-pong [n^3][24] bf16
  DevBuf f;                                 // oct-major f64 source term
  DevBuf wpk_fwd[3], wpk_bwd[3];            // packed B fragments of the hidden layers
  DevBuf wpk_out, wpk_dx;                   // ... of the last layer and of the first layer's input gradient
  DevBuf wpk_xm[3];                         // ... of the hidden layers for the x-marching forward
  DevBuf wpk_out1m;                         // packed B fragments of the last layer, x-planes as columns
  DevBuf wpk_in1;                           // packed B fragments of the first layer
  DevBuf corr_part, red_part, scal;
  int corr_wg = 0;
  double* hp = nullptr;                     // pinned host scalars
  // the packed fragments above match params until params change (set,
  // Adam step); they were written on pack_stream, which pack_ev follows
  bool packed = false;
  hipStream_t pack_stream = nullptr;
  hipEvent_t pack_ev = nullptr;
  ~mgnn_s() {
    if (hp) (void)hipHostFree(hp);
    if (pack_ev) (void)hipEventDestroy(pack_ev);
  }

  void ensure(int nn) {
    if (nn <= n) return;
    const size_t np = (size_t)nn * nn * nn;
    xb.alloc(np * 2);
    xf.alloc(np * 4);
    y.alloc(np * 4);
    t.alloc(np * 4);
    dy.alloc(np * 4);
    dyb.alloc(np * 2);
    for (int l = 0; l < 4; ++l) {
      Z[l].alloc(np * kC * 2);
      A[l].alloc(np * kC * 2);
    }
    G[0].alloc(np * kC * 2);
    G[1].alloc(np * kC * 2);
    f.alloc(std::min<size_t>(np, 16 * 16 * 16) * 8);   // stored only below 32^3 (prepare_input)
    const int64_t tiles = (int64_t)(nn / CX) * (nn / TY) * (nn / TZ);
    corr_wg = (int)std::min<int64_t>(tiles, 1024);
    corr_part.alloc((size_t)corr_wg * kC * kC * kTaps * 4);
    red_part.alloc((size_t)std::max<int64_t>(partial_count((int64_t)np, kReduceBlock), 4096) * 8 * 4);
    n = nn;
  }
};

namespace {

int check_n(int32_t n) {
  MG_REQUIRE(is_pow2(n) && n >= 8 && n <= 1024, "mgnn: n must be a power of two in [8, 1024]");
  return ilog2(n);
}

void pack_weights(mgnn_s* net, hipStream_t s) {
  if (net->packed) {   // packed earlier: a pass on another stream waits for that packing
    if (s != net->pack_stream) MG_HIP(hipStreamWaitEvent(s, net->pack_ev, 0));
    return;
  }
  for (int l = 1; l <= 3; ++l) {
    const float* W = net->params.as<float>() + w_off(l);
    hipLaunchKernelGGL(k_pack24, dim3(blocks_for(kPackVecs)), dim3(256), 0, s, W, net->wpk_fwd[l - 1].as<uint4>(), 0,
                       kC);
    hipLaunchKernelGGL(k_pack24, dim3(blocks_for(kPackVecs)), dim3(256), 0, s, W, net->wpk_bwd[l - 1].as<uint4>(), 1,
                       kC);
  }
  for (int l = 1; l <= 3; ++l)
    hipLaunchKernelGGL(k_pack_xmarch, dim3(blocks_for(kXPackVecs + kXPairVecs)), dim3(256), 0, s,
                       net->params.as<float>() + w_off(l), net->wpk_xm[l - 1].as<uint4>());
  const float* P = net->params.as<float>();
  hipLaunchKernelGGL(k_pack_in1, dim3(1), dim3(128), 0, s, P + w_off(0), net->wpk_in1.as<uint4>());
  hipLaunchKernelGGL(k_pack_out1_mfma, dim3(blocks_for(kO1PackVecs)), dim3(256), 0, s, P + w_off(4),
                     net->wpk_out1m.as<uint4>());
  hipLaunchKernelGGL(k_pack24, dim3(blocks_for(kPackVecs)), dim3(256), 0, s, P + w_off(4), net->wpk_out.as<uint4>(), 0,
                     1);
  hipLaunchKernelGGL(k_pack24, dim3(blocks_for(kPackVecs)), dim3(256), 0, s, P + w_off(0), net->wpk_dx.as<uint4>(), 1,
                     1);
  check_launch();
  if (!net->pack_ev) MG_HIP(hipEventCreateWithFlags(&net->pack_ev, hipEventDisableTiming));
  MG_HIP(hipEventRecord(net->pack_ev, s));
  net->pack_stream = s;
  net->packed = true;
}

// forward on net->xb (the BF16 network input): activations in Z/A, output in net->y
void forward_core(mgnn_s* net, int lg, bool keep_z, hipStream_t s) {
  const int n = 1 << lg;
  const unsigned tiles = (unsigned)((n / TX) * (n / TY) * (n / TZ));
  const float* P = net->params.as<float>();
  pack_weights(net, s);
  bf16_t* z0 = keep_z ? net->Z[0].as<bf16_t>() : nullptr;
  hipLaunchKernelGGL(k_conv_in1_mfma, dim3((unsigned)((n / QX) * (n / QY) * (n / QZ))), dim3(256), 0, s, lg,
                     net->xb.as<bf16_t>(), net->wpk_in1.as<uint4>(), P + b_off(0), z0, net->A[0].as<bf16_t>());
  for (int l = 1; l <= 3; ++l) {
    bf16_t* zl = keep_z ? net->Z[l].as<bf16_t>() : nullptr;
    if (lg >= 5)   // 32^3 and up: the x-marching form
      conv24_xmarch_launch(lg, net->A[l - 1].as<bf16_t>(), net->wpk_xm[l - 1].as<uint4>(), P + b_off(l), zl,
                           net->A[l].as<bf16_t>(), s);
    else
      conv24_launch<0>(lg, net->A[l - 1].as<bf16_t>(), net->wpk_fwd[l - 1].as<uint4>(), P + b_off(l), nullptr, zl,
                       net->A[l].as<bf16_t>(), (float*)nullptr, s);
  }
  if (lg >= 5)
    conv_out1_mfma_launch(lg, net->A[3].as<bf16_t>(), net->wpk_out1m.as<uint4>(), P + b_off(4), net->y.as<float>(), s);
  else
    conv24_launch<2>(lg, net->A[3].as<bf16_t>(), net->wpk_out.as<uint4>(), P + b_off(4), nullptr, nullptr, nullptr,
                     net->y.as<float>(), s);
  check_launch();
}

void weight_grad(mgnn_s* net, int lg, const bf16_t* U, const bf16_t* V, int cv, float* grad_w, int flip, hipStream_t s) {
  const int n = 1 << lg;
  const int64_t tiles = (int64_t)(n / CX) * (n / TY) * (n / TZ);
  const int nwg = (int)std::min<int64_t>(tiles, net->corr_wg);
  if (cv == kC) hipLaunchKernelGGL((k_corr<kC>), dim3(nwg), dim3(256), 0, s, lg, U, V, net->corr_part.as<float>());
  else hipLaunchKernelGGL((k_corr<1>), dim3(nwg), dim3(256), 0, s, lg, U, V, net->corr_part.as<float>());
  const int size = kC * cv * kTaps;
  hipLaunchKernelGGL(k_reduce_partials, dim3(blocks_for(size)), dim3(256), 0, s, net->corr_part.as<float>(), nwg, size,
                     flip, grad_w);
  check_launch();
}

void bias_grad24(mgnn_s* net, int lg, const bf16_t* g, float* grad_b, hipStream_t s) {
  const int64_t np = (int64_t)1 << (3 * lg);
  const int nwg = (int)std::min<int64_t>(1024, (np + 2559) / 2560);
  hipLaunchKernelGGL(k_colsum24, dim3(nwg), dim3(256), 0, s, np, g, net->red_part.as<float>());
  hipLaunchKernelGGL(k_reduce_bias, dim3(1), dim3(64), 0, s, net->red_part.as<float>(), nwg, kC, grad_b);
  check_launch();
}

// backward from net->dy (f32): accumulates parameter gradients; optional dL/dx
void backward_core(mgnn_s* net, int lg, float* dx, hipStream_t s) {
  const int n = 1 << lg;
  const int64_t np = (int64_t)n * n * n;
  const unsigned tiles = (unsigned)((n / TX) * (n / TY) * (n / TZ));
  const float* P = net->params.as<float>();
  float* Gd = net->grads.as<float>();
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(blocks_for(np)), dim3(256), 0, s, np, net->dy.as<float>(),
                     net->dyb.as<bf16_t>(), nullptr);
  // last layer: dW4[0][c][t] = sum_q dy[q] A3[q + t][c] = sum_p A3[p][c] dy[p - t]  (flipped taps)
  weight_grad(net, lg, net->A[3].as<bf16_t>(), net->dyb.as<bf16_t>(), 1, Gd + w_off(4), 1, s);
  {
    const int nwg = (int)std::min<int64_t>(1024, (np + 255) / 256);
    hipLaunchKernelGGL(k_sum_f32, dim3(nwg), dim3(256), 0, s, np, net->dy.as<float>(), net->red_part.as<float>());
    hipLaunchKernelGGL(k_reduce_bias, dim3(1), dim3(64), 0, s, net->red_part.as<float>(), nwg, 1, Gd + b_off(4));
  }
  // dZ3 = conv(dy, W4 flipped) * gelu'(Z3)
  bf16_t* g_cur = net->G[0].as<bf16_t>();
  bf16_t* g_nxt = net->G[1].as<bf16_t>();
  hipLaunchKernelGGL(k_conv_in1_grad, dim3(tiles), dim3(256), 0, s, lg, net->dy.as<float>(), P + w_off(4),
                     net->Z[3].as<bf16_t>(), g_cur);
  for (int l = 3; l >= 1; --l) {
    weight_grad(net, lg, g_cur, net->A[l - 1].as<bf16_t>(), kC, Gd + w_off(l), 0, s);
    bias_grad24(net, lg, g_cur, Gd + b_off(l), s);
    conv24_launch<1>(lg, g_cur, net->wpk_bwd[l - 1].as<uint4>(),
                       nullptr, net->Z[l - 1].as<bf16_t>(), g_nxt, nullptr, (float*)nullptr, s);
    std::swap(g_cur, g_nxt);
  }
  weight_grad(net, lg, g_cur, net->xb.as<bf16_t>(), 1, Gd + w_off(0), 0, s);
  bias_grad24(net, lg, g_cur, Gd + b_off(0), s);
  if (dx)
    conv24_launch<2>(lg, g_cur, net->wpk_dx.as<uint4>(), nullptr,
                       nullptr, nullptr, nullptr, dx, s);
  check_launch();
}

// f = c (rho - mean), sum f^2 -> scal[1]; network input x
void prepare_input(mgnn_s* net, int lg, const double* rho, double rho_mean, double c, hipStream_t s) {
  const int n = 1 << lg;
  const int64_t np = (int64_t)n * n * n;
  double* sc = net->scal.as<double>();
  double* parts = net->red_part.as<double>();
  if (std::isnan(rho_mean)) {
    reduce_final(parts, partial_sum(np, rho, parts, s), 1.0 / (double)np, sc, 0, s);
  } else {
    MG_REQUIRE(std::isfinite(rho_mean), "mgnn: rho_mean must be finite or NAN");
    MG_HIP(hipStreamSynchronize(s));
    net->hp[0] = rho_mean;
    MG_HIP(hipMemcpyAsync(sc, net->hp, sizeof(double), hipMemcpyHostToDevice, s));
  }
  // from 32^3 up the layout transform forms f itself (only ||f||^2 is summed here)
  reduce_final(parts, u_rhs(np, rho, sc, c, lg >= 5 ? nullptr : net->f.as<double>(), parts, s), 1.0, sc, 1, s);
  if (lg >= 5)
    hipLaunchKernelGGL(k_io_tiled, dim3(io_tiles(lg)), dim3(256), 0, s, lg, 0, sc, c, rho, nullptr, nullptr,
                       net->xf.as<float>(), net->xb.as<bf16_t>());
  else
    hipLaunchKernelGGL(k_input, dim3(blocks_for(np)), dim3(256), 0, s, lg, net->f.as<double>(), sc,
                       net->xb.as<bf16_t>(), net->xf.as<float>());
  check_launch();
}

void init_params_host(std::vector<float>& p, uint64_t seed) {
  // splitmix64 -> uniform -> Box-Muller normal; He-normal std sqrt(2 / (27 c_in))
  uint64_t st = seed;
  auto next = [&]() {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto uni = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
  auto normal = [&]() { return std::sqrt(-2.0 * std::log(uni())) * std::cos(2.0 * M_PI * uni()); };
  p.assign(kNumParams, 0.f);
  const int cin[5] = {1, kC, kC, kC, kC};
  const int cout[5] = {kC, kC, kC, kC, 1};
  for (int l = 0; l < 5; ++l) {
    const double std_ = std::sqrt(2.0 / (27.0 * cin[l]));
    for (int i = 0; i < cout[l] * cin[l] * kTaps; ++i) p[w_off(l) + i] = (float)(normal() * std_);
  }
}

}  // namespace

extern "C" {

mg_status_t mgnn_create(int32_t channels, int32_t layers, uint64_t seed, mgnn_t* out) {
  MG_API_BEGIN
  MG_REQUIRE(out != nullptr, "mgnn_create: out is NULL");
  *out = nullptr;
  MG_REQUIRE(channels == kC && layers == 5, "mgnn_create: only 24 channels and 5 layers are supported");
  std::unique_ptr<mgnn_s> net(new mgnn_s());
  net->params.alloc(kNumParams * 4);
  net->grads.alloc(kNumParams * 4);
  net->adam_m.alloc(kNumParams * 4);
  net->adam_v.alloc(kNumParams * 4);
  for (int l = 0; l < 3; ++l) {
    net->wpk_fwd[l].alloc(kPackVecs * 16);
    net->wpk_xm[l].alloc((kXPackVecs + kXPairVecs) * 16);
    net->wpk_bwd[l].alloc(kPackVecs * 16);
  }
  net->wpk_out.alloc(kPackVecs * 16);
  net->wpk_dx.alloc(kPackVecs * 16);
  net->wpk_out1m.alloc(kO1PackVecs * 16);
  net->wpk_in1.alloc(2 * 64 * 16);
  net->scal.alloc(8 * sizeof(double));
  MG_HIP(hipHostMalloc((void**)&net->hp, 8 * sizeof(double), hipHostMallocDefault));
  std::vector<float> p;
  init_params_host(p, seed);
  MG_HIP(hipMemcpy(net->params.p, p.data(), kNumParams * 4, hipMemcpyHostToDevice));
  MG_HIP(hipMemset(net->grads.p, 0, kNumParams * 4));
  MG_HIP(hipMemset(net->adam_m.p, 0, kNumParams * 4));
  MG_HIP(hipMemset(net->adam_v.p, 0, kNumParams * 4));
  *out = net.release();
  return MG_OK;
  MG_API_END
}

void mgnn_destroy(mgnn_t net) { delete net; }

int64_t mgnn_num_params(mgnn_t net) { return net ? kNumParams : 0; }

mg_status_t mgnn_get_weights(mgnn_t net, float* h_buf, int64_t n) {
  MG_API_BEGIN
  MG_REQUIRE(net && h_buf && n == kNumParams, "mgnn_get_weights: bad argument (n must equal mgnn_num_params)");
  MG_HIP(hipDeviceSynchronize());
  MG_HIP(hipMemcpy(h_buf, net->params.p, kNumParams * 4, hipMemcpyDeviceToHost));
  return MG_OK;
  MG_API_END
}

mg_status_t mgnn_set_weights(mgnn_t net, const float* h_buf, int64_t n) {
  MG_API_BEGIN
  MG_REQUIRE(net && h_buf && n == kNumParams, "mgnn_set_weights: bad argument (n must equal mgnn_num_params)");
  MG_HIP(hipDeviceSynchronize());
  MG_HIP(hipMemcpy(net->params.p, h_buf, kNumParams * 4, hipMemcpyHostToDevice));
  net->packed = false;
  return MG_OK;
  MG_API_END
}

mg_status_t mgnn_get_grads(mgnn_t net, float* h_buf, int64_t n) {
  MG_API_BEGIN
  MG_REQUIRE(net && h_buf && n == kNumParams, "mgnn_get_grads: bad argument (n must equal mgnn_num_params)");
  MG_HIP(hipDeviceSynchronize());
  MG_HIP(hipMemcpy(h_buf, net->grads.p, kNumParams * 4, hipMemcpyDeviceToHost));
  return MG_OK;
  MG_API_END
}

mg_status_t mgnn_zero_grad(mgnn_t net, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(net != nullptr, "mgnn_zero_grad: NULL handle");
  fill_zero<float>(net->grads.as<float>(), kNumParams, (hipStream_t)stream);
  return MG_OK;
  MG_API_END
}

mg_status_t mgnn_forward_raw(mgnn_t net, int32_t n, const float* d_x, float* d_y, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(net && d_x && d_y, "mgnn_forward_raw: NULL argument");
  const int lg = check_n(n);
  hipStream_t s = (hipStream_t)stream;
  net->ensure(n);
  const int64_t np = (int64_t)n * n * n;
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(blocks_for(np)), dim3(256), 0, s, np, d_x, net->xb.as<bf16_t>(),
                     net->xf.as<float>());
  check_launch();
  forward_core(net, lg, true, s);
  net->field_n = 0;
  MG_HIP(hipMemcpyAsync(d_y, net->y.p, np * 4, hipMemcpyDeviceToDevice, s));
  return MG_OK;
  MG_API_END
}

mg_status_t mgnn_backward_raw(mgnn_t net, int32_t n, const float* d_dy, float* d_dx, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(net && d_dy, "mgnn_backward_raw: NULL argument");
  const int lg = check_n(n);
  MG_REQUIRE(net->n >= n, "mgnn_backward_raw: no forward pass at this size");
  hipStream_t s = (hipStream_t)stream;
  const int64_t np = (int64_t)n * n * n;
  MG_HIP(hipMemcpyAsync(net->dy.p, d_dy, np * 4, hipMemcpyDeviceToDevice, s));
  backward_core(net, lg, d_dx, s);
  return MG_OK;
  MG_API_END
}

mg_status_t mgnn_backward(mgnn_t net, int32_t n, const float* d_dloss_dphi, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(net && d_dloss_dphi, "mgnn_backward: NULL argument");
  const int lg = check_n(n);
  MG_REQUIRE(net->field_n == n, "mgnn_backward: the last pass of this handle was not an mgnn_forward at this n");
  hipStream_t s = (hipStream_t)stream;
  const int64_t np = (int64_t)n * n * n;
  // mgnn_forward keeps only its input: the activations are recomputed here
  forward_core(net, lg, true, s);
  hipLaunchKernelGGL(k_dphi_to_dy, dim3(blocks_for(np)), dim3(256), 0, s, lg, net->scal.as<double>(), d_dloss_dphi,
                     net->dy.as<float>());
  check_launch();
  backward_core(net, lg, nullptr, s);
  return MG_OK;
  MG_API_END
}

mg_status_t mgnn_adam_step(mgnn_t net, float lr, float b1, float b2, float eps, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(net != nullptr, "mgnn_adam_step: NULL handle");
  MG_REQUIRE(lr >= 0.f && b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f && eps > 0.f, "mgnn_adam_step: bad hyper-parameters");
  net->step += 1;
  const float bc1 = 1.f - std::pow(b1, (float)net->step), bc2 = 1.f - std::pow(b2, (float)net->step);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(kNumParams)), dim3(256), 0, (hipStream_t)stream, kNumParams,
                     net->params.as<float>(), net->grads.as<float>(), net->adam_m.as<float>(), net->adam_v.as<float>(),
                     lr, b1, b2, eps, bc1, bc2);
  check_launch();
  net->packed = false;
  return MG_OK;
  MG_API_END
}

mg_status_t mgnn_forward(mgnn_t net, int32_t n, const double* d_rho, double rho_mean, double four_pi_G,
                         double* d_phi0, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(net && d_rho && d_phi0, "mgnn_forward: NULL argument");
  MG_REQUIRE(std::isfinite(four_pi_G), "mgnn_forward: four_pi_G must be finite");
  const int lg = check_n(n);
  hipStream_t s = (hipStream_t)stream;
  net->ensure(n);
  const int64_t np = (int64_t)n * n * n;
  prepare_input(net, lg, d_rho, rho_mean, four_pi_G, s);
  forward_core(net, lg, false, s);
  net->field_n = n;
  if (lg >= 5)
    hipLaunchKernelGGL(k_io_tiled, dim3(io_tiles(lg)), dim3(256), 0, s, lg, 1, net->scal.as<double>(), 0.0, nullptr,
                       net->y.as<float>(), d_phi0, nullptr, nullptr);
  else
    hipLaunchKernelGGL(k_scale_io, dim3(blocks_for(np)), dim3(256), 0, s, lg, 0, net->scal.as<double>(),
                       net->y.as<float>(), d_phi0, nullptr, nullptr);
  check_launch();
  return MG_OK;
  MG_API_END
}

mg_status_t mgnn_train_step(mgnn_t net, int32_t n, const double* d_rho, double rho_mean, double four_pi_G,
                            const double* d_phi_target, float lr, float res_weight, double* h_loss, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(net && d_rho && d_phi_target, "mgnn_train_step: NULL argument");
  MG_REQUIRE(std::isfinite(four_pi_G) && lr >= 0.f && res_weight >= 0.f, "mgnn_train_step: bad argument");
  const int lg = check_n(n);
  hipStream_t s = (hipStream_t)stream;
  net->ensure(n);
  const int64_t np = (int64_t)n * n * n;
  prepare_input(net, lg, d_rho, rho_mean, four_pi_G, s);
  net->field_n = 0;
  if (lg >= 5)
    hipLaunchKernelGGL(k_io_tiled, dim3(io_tiles(lg)), dim3(256), 0, s, lg, 2, net->scal.as<double>(), 0.0, d_phi_target,
                       nullptr, nullptr, net->t.as<float>(), nullptr);
  else
    hipLaunchKernelGGL(k_scale_io, dim3(blocks_for(np)), dim3(256), 0, s, lg, 1, net->scal.as<double>(), nullptr,
                       nullptr, d_phi_target, net->t.as<float>());
  forward_core(net, lg, true, s);
  const int nwg = (int)std::min<int64_t>(1024, (np + 255) / 256);
  hipLaunchKernelGGL(k_sumsq, dim3(nwg), dim3(256), 0, s, np, net->t.as<float>(), net->red_part.as<double>());
  reduce_final(net->red_part.as<double>(), nwg, 1.0, net->scal.as<double>(), 4, s);
  hipLaunchKernelGGL(k_mse, dim3(nwg), dim3(256), 0, s, np, net->y.as<float>(), net->t.as<float>(),
                     net->scal.as<double>() + 4, net->dy.as<float>(), net->red_part.as<double>());
  reduce_final(net->red_part.as<double>(), nwg, 1.0, net->scal.as<double>(), 2, s);
  if (res_weight > 0.f) {
    // t is consumed; reuse it for R
    hipLaunchKernelGGL(k_res_r, dim3(nwg), dim3(256), 0, s, lg, net->xf.as<float>(), net->y.as<float>(), net->t.as<float>(),
                       net->red_part.as<double>());
    reduce_final(net->red_part.as<double>(), nwg, (double)res_weight / (double)np, net->scal.as<double>(), 3, s);
    hipLaunchKernelGGL(k_res_dy, dim3(blocks_for(np)), dim3(256), 0, s, lg, net->t.as<float>(), res_weight,
                       net->dy.as<float>());
    check_launch();
  } else {
    fill_zero<double>(net->scal.as<double>() + 3, 1, s);
  }
  fill_zero<float>(net->grads.as<float>(), kNumParams, s);
  backward_core(net, lg, nullptr, s);
  MG_HIP(hipMemcpyAsync(net->hp + 2, net->scal.as<double>() + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  net->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - std::pow(b1, (float)net->step), bc2 = 1.f - std::pow(b2, (float)net->step);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(kNumParams)), dim3(256), 0, s, kNumParams, net->params.as<float>(),
                     net->grads.as<float>(), net->adam_m.as<float>(), net->adam_v.as<float>(), lr, b1, b2, 1e-8f, bc1,
                     bc2);
  check_launch();
  net->packed = false;
  MG_HIP(hipStreamSynchronize(s));
  if (h_loss) *h_loss = net->hp[2] + net->hp[3];
  return MG_OK;
  MG_API_END
}

mg_status_t mgnn_solve_warm(mgnn_t net, mg_level_t L, const double* d_rho, double rho_mean, double four_pi_G,
                            double* d_phi, double tol, int32_t max_cycles, mg_solve_info_t* info,
                            int32_t* used_fallback) {
  MG_API_BEGIN
  MG_REQUIRE(net && L && d_rho && d_phi, "mgnn_solve_warm: NULL argument");
  MG_REQUIRE(L->periodic, "mgnn_solve_warm: the warm start is defined on the periodic base level");
  MG_REQUIRE(tol > 0.0 && max_cycles >= 0 && std::isfinite(four_pi_G) && four_pi_G != 0.0, "mgnn_solve_warm: bad argument");
  hipStream_t s = L->stream;
  hipEvent_t e0, e1;
  MG_HIP(hipEventCreate(&e0));
  MG_HIP(hipEventCreate(&e1));
  MG_HIP(hipEventRecord(e0, s));
  MG_REQUIRE(mgnn_forward(net, L->n, d_rho, rho_mean, four_pi_G, d_phi, s) == MG_OK, get_error());
  double rn = 0.0, fn = 0.0;
  L->residual_norm(d_rho, rho_mean, four_pi_G, nullptr, d_phi, rn, fn);
  const bool bad = !(std::isfinite(rn) && std::isfinite(fn) && fn > 0.0 && rn < fn);
  if (bad) fill_zero<double>(d_phi, L->n_cells, s);
  if (used_fallback) *used_fallback = bad ? 1 : 0;
  mg_solve_info_t tmp{};
  const mg_status_t st = L->solve(d_rho, rho_mean, four_pi_G, nullptr, d_phi, tol, max_cycles, tmp);
  tmp.used_fallback = bad ? 1 : 0;
  MG_HIP(hipEventRecord(e1, s));
  MG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  MG_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tmp.ms = ms;
  if (!bad && fn > 0.0) tmp.relres0 = rn / fn;
  if (info) *info = tmp;
  return st;
  MG_API_END
}

}  // extern "C"

// Kernels on a full periodic level (n^3 cells, oct-major, octs lexicographic).
//
// Cell c = cx + 2cy + 4cz of oct (ox, oy, oz) sits at (2ox+cx, 2oy+cy, 2oz+cz).
// Its face neighbour along axis d is cell c ^ (1 << d): inside the same oct,
// or (same index) inside the adjacent oct on the side given by bit d of c --
// the low side when the bit is 0, the high side when it is 1.  Colour
// (i + j + k) mod 2 of a cell equals the parity of cx + cy + cz because octs sit
// at even offsets; red = 0 is updated first.
#include <type_traits>

#include "mg_internal.h"

namespace mg {

namespace {

constexpr int kBlock = 256;

struct OctGeom {
  int lno;       // log2(octs per dimension)
  int m;         // octs per dimension - 1
  __device__ __forceinline__ int64_t idx(int x, int y, int z) const {
    return ((((int64_t)(z & m) << lno) + (y & m)) << lno) + (x & m);
  }
};

__device__ __forceinline__ constexpr int colour_of(int c) { return (c ^ (c >> 1) ^ (c >> 2)) & 1; }

template <typename T>
__device__ __forceinline__ void load8(const T* __restrict__ p, T (&v)[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = p[c];
}

// Sum of the six face neighbours of cell c of the oct whose values are `own`;
// nb[j] are the neighbour oct indices in directions -x,+x,-y,+y,-z,+z.
template <typename T>
__device__ __forceinline__ T nbr_sum(const T* __restrict__ a, const T (&own)[8], const int64_t (&nb)[6], int c) {
  T s = own[c ^ 1] + own[c ^ 2] + own[c ^ 4];
  s += a[nb[(c & 1) ? 1 : 0] * 8 + (c ^ 1)];
  s += a[nb[(c & 2) ? 3 : 2] * 8 + (c ^ 2)];
  s += a[nb[(c & 4) ? 5 : 4] * 8 + (c ^ 4)];
  return s;
}

__device__ __forceinline__ void oct_coords(int64_t o, int lno, int m, int& ox, int& oy, int& oz) {
  ox = (int)(o & m);
  oy = (int)((o >> lno) & m);
  oz = (int)(o >> (2 * lno));
}

// ---- red-black Gauss-Seidel half sweep (equation gs_update) ---------------
template <typename T, int COLOUR>
__global__ __launch_bounds__(kBlock) void k_smooth_colour(int lno, T h2, T* __restrict__ phi,
                                                          const T* __restrict__ b) {
  const int64_t n_oct = (int64_t)1 << (3 * lno);
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_oct) return;
  const OctGeom g{lno, (1 << lno) - 1};
  int ox, oy, oz;
  oct_coords(o, lno, g.m, ox, oy, oz);
  const int64_t nb[6] = {g.idx(ox - 1, oy, oz), g.idx(ox + 1, oy, oz), g.idx(ox, oy - 1, oz),
                         g.idx(ox, oy + 1, oz), g.idx(ox, oy, oz - 1), g.idx(ox, oy, oz + 1)};
  T own[8];
  load8(phi + o * 8, own);
  const T sixth = T(1) / T(6);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (colour_of(c) != COLOUR) continue;
    const T s = nbr_sum(phi, own, nb, c);
    phi[o * 8 + c] = (s - h2 * b[o * 8 + c]) * sixth;
  }
}

// ---- fused red + black sweep on an LDS tile ---------------------------------
// One workgroup owns a tile of 16 x 16 x 8 cells (8 x 8 x 4 octs, one oct per
// thread).  It stages phi of the tile plus a one-oct halo (20 x 20 x 12 cells)
// in LDS as a dense cell grid, updates the red cells of the tile and of the
// one-cell shell around it (the shell's red values are exactly what the
// neighbouring tiles compute, since they depend only on black values that no
// one has changed yet), then the black cells of the tile, and writes the tile
// back: one read of phi and b and one write of phi per cell and sweep.  The
// sweep reads `src` and writes `dst` (two buffers), so a halo is never read
// after its owner has written it: the result is exactly the red-then-black
// Gauss-Seidel sweep, independent of workgroup timing.  Tiles are assigned
// XCD by XCD so that neighbouring tiles share an L2.
constexpr int kTX = 16, kTY = 16, kTZ = 8;                       // tile, cells
constexpr int kLX = kTX + 4, kLY = kTY + 4, kLZ = kTZ + 4;       // LDS box, cells
constexpr int kRX = kTX / 2 + 2, kRY = kTY / 2 + 2, kRZ = kTZ / 2 + 2;   // LDS box, octs
constexpr int kTileThreads = (kTX / 2) * (kTY / 2) * (kTZ / 2);  // one thread per interior oct

__host__ __device__ constexpr int lds_idx(int x, int y, int z) { return (z * kLY + y) * kLX + x; }

// the red cells of the one-cell shell around the tile, as LDS indices
constexpr int kShellRed = ((kTX + 2) * (kTY + 2) * (kTZ + 2) - kTX * kTY * kTZ) / 2;
struct ShellTable {
  uint16_t v[kShellRed];
};
constexpr ShellTable make_shell_table() {
  ShellTable t{};
  int k = 0;
  for (int z = 1; z < kLZ - 1; ++z)
    for (int y = 1; y < kLY - 1; ++y)
      for (int x = 1; x < kLX - 1; ++x) {
        const bool inner = x >= 2 && x < kLX - 2 && y >= 2 && y < kLY - 2 && z >= 2 && z < kLZ - 2;
        if (!inner && ((x + y + z) & 1) == 0) t.v[k++] = (uint16_t)lds_idx(x, y, z);
      }
  return t;
}
__constant__ ShellTable kShell = make_shell_table();
constexpr int kShellPerThread = (kShellRed + kTileThreads - 1) / kTileThreads;

// 16-byte vector of T
template <typename T> struct Vec16;
template <> struct Vec16<double> { using type = double2; static constexpr int n = 2; };
template <> struct Vec16<float> { using type = float4; static constexpr int n = 4; };

// With `partials` set, the kernel also adds up ||b - L phi||^2 of the incoming
// phi over the tile's cells (f64, from the staged LDS values, before any
// update) and writes one partial sum per tile.
// PROLONG: the sweep applies to phi + P ec, the trilinear prolongation of the
// coarse correction ec (grid n/2), added to every staged cell; the coarse
// cells the box needs (12 x 12 x 8) are staged first.
// ZERO: the incoming phi is zero; it is not read (the first sweep from a zero
// guess reads only b).  With `add64` (f64, same layout) the swept values are
// added to add64 instead of being written to dst: the last sweep of an FP32
// correction cycle applies the correction to the FP64 iterate directly.
constexpr int kCX = kLX / 2 + 2, kCY = kLY / 2 + 2, kCZ = kLZ / 2 + 2;   // coarse box, cells
template <typename T, bool PROLONG, bool ZERO>
__global__ __launch_bounds__(kTileThreads) void k_smooth_tile(int lno, T h2, const T* __restrict__ phi,
                                                              const T* __restrict__ b, T* __restrict__ dst,
                                                              double* __restrict__ partials,
                                                              const T* __restrict__ ec,
                                                              double* __restrict__ add64) {
  static_assert(!(PROLONG && ZERO), "a prolongation needs an incoming phi");
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;            // values per 16-byte vector
  constexpr int VPO = 8 / VN;                // vectors per oct
  __shared__ T s[kLX * kLY * kLZ];
  __shared__ T sc[PROLONG ? kCX * kCY * kCZ : 1];
  const int n_cell = 2 << lno;                 // cells per dimension
  const int m = (1 << lno) - 1;                // octs per dimension - 1
  const int tnx = n_cell / kTX, tny = n_cell / kTY, tnz = n_cell / kTZ;
  const int nb = tnx * tny * tnz;
  int tile = blockIdx.x;
  if ((nb & 7) == 0) tile = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int tx = tile % tnx, ty = (tile / tnx) % tny, tz = tile / (tnx * tny);
  const int ox0 = tx * (kTX / 2), oy0 = ty * (kTY / 2), oz0 = tz * (kTZ / 2);   // tile origin, octs
  const OctGeom g{lno, m};
  const int t = threadIdx.x;

  // this thread's interior oct and its right-hand side (16-byte loads)
  const int ix = t % (kTX / 2), iy = (t / (kTX / 2)) % (kTY / 2), iz = t / ((kTX / 2) * (kTY / 2));
  const int64_t my_oct = g.idx(ox0 + ix, oy0 + iy, oz0 + iz);
  T bo[8];
  {
    const V* bv = reinterpret_cast<const V*>(b + my_oct * 8);
#pragma unroll
    for (int k = 0; k < VPO; ++k) {
      const V v = bv[k];
      const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
      for (int j = 0; j < VN; ++j) bo[k * VN + j] = pv[j];
    }
  }
  // Every global load of the tile is issued before the first wait: the loops
  // below are unrolled, with indices clamped instead of branched on, so the
  // memory system sees all of a thread's requests at once.
  // right-hand side of this thread's shell cells
  T bs[kShellPerThread];
  int li[kShellPerThread];   // their LDS indices
  {
#pragma unroll
    for (int r = 0; r < kShellPerThread; ++r) li[r] = kShell.v[min(t + r * kTileThreads, kShellRed - 1)];
#pragma unroll
    for (int r = 0; r < kShellPerThread; ++r) {
      const int x = li[r] % kLX, y = (li[r] / kLX) % kLY, z = li[r] / (kLX * kLY);
      const int gx = 2 * ox0 - 2 + x, gy = 2 * oy0 - 2 + y, gz = 2 * oz0 - 2 + z;   // global cell coords
      bs[r] = b[g.idx(gx >> 1, gy >> 1, gz >> 1) * 8 + (gx & 1) + 2 * (gy & 1) + 4 * (gz & 1)];
    }
  }
  // coarse correction box (PROLONG): coarse cells (ox0 - 2, ...) + [0, kC*),
  // i.e. coarse octs (ox0/2 - 1, ...) + [0, kC*/2)
  constexpr int NOX = kCX / 2, NOY = kCY / 2, NOZ = kCZ / 2;
  constexpr int kCoarseVec = NOX * NOY * NOZ * VPO;
  constexpr int kCoarsePer = PROLONG ? (kCoarseVec + kTileThreads - 1) / kTileThreads : 0;
  V cv[kCoarsePer > 0 ? kCoarsePer : 1];
  if (PROLONG) {
    const int lnc = lno - 1, mc = (1 << lnc) - 1;
    const int cox = ox0 / 2 - 1, coy = oy0 / 2 - 1, coz = oz0 / 2 - 1;
#pragma unroll
    for (int r = 0; r < kCoarsePer; ++r) {
      const int q = min(t + r * kTileThreads, kCoarseVec - 1);
      const int o = q / VPO, part = q % VPO;
      const int qx = o % NOX, qy = (o / NOX) % NOY, qz = o / (NOX * NOY);
      const int64_t co = ((((int64_t)((coz + qz) & mc) << lnc) + ((coy + qy) & mc)) << lnc) + ((cox + qx) & mc);
      cv[r] = reinterpret_cast<const V*>(ec + co * 8)[part];
    }
  }
  // phi of the tile plus a one-oct halo: consecutive lanes read consecutive 16-byte pieces
  constexpr int kStageVec = kRX * kRY * kRZ * VPO;
  constexpr int kStagePer = (kStageVec + kTileThreads - 1) / kTileThreads;
  V sv[ZERO ? 1 : kStagePer];
  if (!ZERO) {
#pragma unroll
    for (int r = 0; r < kStagePer; ++r) {
      const int q = min(t + r * kTileThreads, kStageVec - 1);
      const int o = q / VPO, part = q % VPO;
      const int qx = o % kRX, qy = (o / kRX) % kRY, qz = o / (kRX * kRY);
      sv[r] = reinterpret_cast<const V*>(phi + g.idx(ox0 - 1 + qx, oy0 - 1 + qy, oz0 - 1 + qz) * 8)[part];
    }
  }
  if (PROLONG) {
#pragma unroll
    for (int r = 0; r < kCoarsePer; ++r) {
      const int q = t + r * kTileThreads;
      if (q < kCoarseVec) {
        const int o = q / VPO, part = q % VPO;
        const int qx = o % NOX, qy = (o / NOX) % NOY, qz = o / (NOX * NOY);
        const T* pv = reinterpret_cast<const T*>(&cv[r]);
#pragma unroll
        for (int j = 0; j < VN; ++j) {
          const int c = part * VN + j;
          sc[((2 * qz + (c >> 2)) * kCY + 2 * qy + ((c >> 1) & 1)) * kCX + 2 * qx + (c & 1)] = pv[j];
        }
      }
    }
    __syncthreads();
  }
  if (ZERO) {
    for (int q = t; q < kLX * kLY * kLZ; q += kTileThreads) s[q] = T(0);
  }
#pragma unroll
  for (int r = 0; r < (ZERO ? 0 : kStagePer); ++r) {
    const int q = t + r * kTileThreads;
    if (q < kStageVec) {
      const int o = q / VPO, part = q % VPO;
      const int qx = o % kRX, qy = (o / kRX) % kRY, qz = o / (kRX * kRY);
      const T* pv = reinterpret_cast<const T*>(&sv[r]);
#pragma unroll
      for (int j = 0; j < VN; ++j) {
        const int c = part * VN + j;
        const int lx = 2 * qx + (c & 1), ly = 2 * qy + ((c >> 1) & 1), lz = 2 * qz + (c >> 2);
        T val = pv[j];
        if (PROLONG) {
          // parent (1 + l/2 in the coarse box), neighbour on the child's side, weights 3/4 and 1/4 per axis
          const int px = 1 + (lx >> 1), py = 1 + (ly >> 1), pz = 1 + (lz >> 1);
          const int sx = (lx & 1) ? 1 : -1, sy = (ly & 1) ? 1 : -1, sz = (lz & 1) ? 1 : -1;
          const T w[2] = {T(0.75), T(0.25)};
          T corr = T(0);
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb)
#pragma unroll
              for (int cc = 0; cc < 2; ++cc)
                corr += (w[a] * w[bb] * w[cc]) * sc[((pz + cc * sz) * kCY + py + bb * sy) * kCX + px + a * sx];
          val += corr;
        }
        s[lds_idx(lx, ly, lz)] = val;
      }
    }
  }
  __syncthreads();

  const T sixth = T(1) / T(6);
  auto nsum = [&](int i) {
    return s[i - 1] + s[i + 1] + s[i - kLX] + s[i + kLX] + s[i - kLX * kLY] + s[i + kLX * kLY];
  };
  const int i0 = lds_idx(2 * ix + 2, 2 * iy + 2, 2 * iz + 2);   // LDS index of cell 0 of the oct
  auto cell_off = [](int c) { return (c & 1) + ((c >> 1) & 1) * kLX + (c >> 2) * kLX * kLY; };
  if (partials) {
    // residual norm of the incoming phi (uniform branch: `partials` is a kernel argument)
    const T inv_h2 = T(1) / h2;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int i = i0 + cell_off(c);
      const T r = bo[c] - (nsum(i) - T(6) * s[i]) * inv_h2;
      acc += (double)r * (double)r;
    }
    const double tot = block_sum(acc);
    if (t == 0) partials[blockIdx.x] = tot;
    __syncthreads();
  }
  // red: the tile's own octs
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (colour_of(c) != 0) continue;
    const int i = i0 + cell_off(c);
    s[i] = (nsum(i) - h2 * bo[c]) * sixth;
  }
  // red: the one-cell shell around the tile
#pragma unroll
  for (int r = 0; r < kShellPerThread; ++r) {
    if (t + r * kTileThreads < kShellRed) {
      const int i = li[r];
      s[i] = (nsum(i) - h2 * bs[r]) * sixth;
    }
  }
  __syncthreads();
  // black: the tile's own octs, then write the oct back (16-byte stores)
  T out[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int i = i0 + cell_off(c);
    out[c] = colour_of(c) == 0 ? s[i] : (nsum(i) - h2 * bo[c]) * sixth;
  }
  if (add64) {
    // the result is a correction: add it to the f64 iterate instead of storing it
    double2* av = reinterpret_cast<double2*>(add64 + my_oct * 8);
    double2 a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = av[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k].x += (double)out[2 * k];
      a[k].y += (double)out[2 * k + 1];
      av[k] = a[k];
    }
    return;
  }
  V* dv = reinterpret_cast<V*>(dst + my_oct * 8);
#pragma unroll
  for (int k = 0; k < VPO; ++k) {
    V v;
    T* pv = reinterpret_cast<T*>(&v);
#pragma unroll
    for (int j = 0; j < VN; ++j) pv[j] = out[k * VN + j];
    dv[k] = v;
  }
}

// ---- red-black sweep marching along z through an LDS ring ----------------------
// One workgroup owns an xy column of 32 x 16 cells (16 x 8 octs, two
// threads per oct, one per cell plane) and a run of kz oct layers along z.  It streams the layers of its
// box (the column plus a one-oct halo in x and y: 36 x 20 cells) through a
// ring of 8 cell planes (4 oct layers) in LDS, one oct layer per step:
//   A  write layer s-1 (loaded during the previous step) into the ring
//   B  issue the loads of layer s (phi box, own b, b of the shell cells)
//   C  (with `partials`) ||b - L phi||^2 of the incoming phi: lower plane of
//      layer s-1, upper plane of layer s-2 -- both still untouched (a barrier
//      separates these reads from D's writes)
//   D  red update of layer s-2 on the column plus its one-cell xy ring (only
//      the upper plane for layer -1, only the lower for layer kz)
//   E  black update of layer s-3 on the column, which is then final: store it
// Every update reads exactly the values the red-then-black sweep would, so the
// result equals the sequential sweep; the halo is re-read only in x and y and
// at the ends of the run (three extra layers per kz).  Runs are assigned XCD by
// XCD, each XCD's columns marching the same z range together so that their
// shared x/y halos hit in its L2.
constexpr int kMX = 32, kMY = 16;                   // column, cells
constexpr int kMOX = kMX / 2, kMOY = kMY / 2;       // column, octs
constexpr int kMOcts = kMOX * kMOY;                 // 128
// threads per oct: FP64 gives each of an oct's two cell planes its own thread
// (two waves per SIMD hide the LDS latency of the updates); FP32, one thread
// per oct (with half the registers per value, more workgroups fit instead).
// Measured on 256^3: FP64 90 -> 84 us per sweep with two, FP32 35 -> 45 us.
template <typename T> struct March {
  static constexpr int split = sizeof(T) == 8 ? 2 : 1;
  static constexpr int cpt = 8 / split;             // cells per thread
  static constexpr int threads = kMOcts * split;
};
constexpr int kMBX = kMX + 4, kMBY = kMY + 4;       // box, cells
constexpr int kMBOX = kMBX / 2, kMBOY = kMBY / 2;   // box, octs
constexpr int kMPlane = kMBX * kMBY;                // cells per LDS plane
constexpr int kMShell = ((kMX + 2) * (kMY + 2) - kMX * kMY);   // red cells of the xy ring in one oct layer
struct MarchShell {
  uint16_t v[kMShell];   // lx | ly << 6 | plane << 12
};
constexpr MarchShell make_march_shell() {
  MarchShell t{};
  int k = 0;
  for (int p = 0; p < 2; ++p)
    for (int y = 1; y < kMBY - 1; ++y)
      for (int x = 1; x < kMBX - 1; ++x) {
        const bool inner = x >= 2 && x < kMBX - 2 && y >= 2 && y < kMBY - 2;
        if (!inner && ((x + y + p) & 1) == 0) t.v[k++] = (uint16_t)(x | (y << 6) | (p << 12));
      }
  return t;
}
__constant__ MarchShell kMarchShell = make_march_shell();

// PROLONG: the sweep applies to phi + P ec (trilinear prolongation of the
// coarse correction ec on the grid n/2).  The coarse planes a layer needs
// (20 x 12 coarse cells each) are held in registers, three at a time; as a
// layer enters the ring, its two z-interpolated coarse planes (one per cell
// plane of the layer) go to LDS, and each 16-byte piece of the layer then
// interpolates in y and x from a 3 x 2 (FP64: two cells along x) or 3 x 3
// (FP32: 2 x 2 cells) window of them.
constexpr int kMCX = kMBX / 2 + 2, kMCY = kMBY / 2 + 2;   // coarse plane, cells (20 x 12)
constexpr int kMCPlane = kMCX * kMCY;
template <typename T, bool ZERO, bool PROLONG>
__global__ __launch_bounds__(March<T>::threads) void k_smooth_march(int lno, int chunks, T h2, const T* __restrict__ phi,
                                                            const T* __restrict__ b, T* __restrict__ dst,
                                                            double* __restrict__ partials,
                                                            double* __restrict__ add64, const T* __restrict__ ec) {
  static_assert(!(PROLONG && ZERO), "a prolongation needs an incoming phi");
  constexpr int kMSplit = March<T>::split, kMCPT = March<T>::cpt, kMThreads = March<T>::threads;
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  constexpr int VPO = 8 / VN;
  constexpr int kVec = kMBOX * kMBOY * VPO;                  // 16-byte pieces of one box layer
  constexpr int kPF = (kVec + kMThreads - 1) / kMThreads;
  __shared__ T s[8 * kMPlane];
  __shared__ T zc[PROLONG ? 2 * kMCPlane : 1];
  const int m = (1 << lno) - 1;
  const int n_cell = 2 << lno;
  const int ncx = n_cell / kMX, cols = ncx * (n_cell / kMY);
  const int nb = cols * chunks;
  int u = blockIdx.x;
  if ((nb & 7) == 0) u = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int col = u % cols, chunk = u / cols;
  const int ox0 = (col % ncx) * kMOX, oy0 = (col / ncx) * kMOY;
  const int oz0 = (chunk << lno) / chunks;                 // this run's oct layers: [oz0, oz0 + kz)
  const int kz = ((chunk + 1) << lno) / chunks - oz0;
  const OctGeom g{lno, m};
  const int t = threadIdx.x;
  const int to = t % kMOcts, hz = kMSplit == 1 ? 0 : t / kMOcts;   // own oct, own cell plane (wave-uniform)
  const int ix = to % kMOX, iy = to / kMOX;
  auto cell = [&](int j) { return kMSplit == 1 ? j : 4 * hz + j; };   // oct cell of the thread's j-th cell
  int slx = 0, sly = 0, sp = 0;
  if (t < kMShell) {
    const int v = kMarchShell.v[t];
    slx = v & 63;
    sly = (v >> 6) & 63;
    sp = v >> 12;
  }
  const T sixth = T(1) / T(6);
  const T inv_h2 = T(1) / h2;
  V pf[kPF];
  T bo[4][kMCPT];   // b of the own cells, one slot per layer in flight (layer j in slot j & 3)
  T bs[4];      // b of this thread's shell cell, same slots
  double acc = 0.0;

  auto plane_of = [](int j, int cz) { return (2 * j + cz + 8) & 7; };
  auto nsum = [&](int P, int xy) {
    const int i = P * kMPlane + xy;
    return s[i - 1] + s[i + 1] + s[i - kMBX] + s[i + kMBX] + s[((P + 7) & 7) * kMPlane + xy] +
           s[((P + 1) & 7) * kMPlane + xy];
  };
  auto own_xy = [&](int c) { return (2 + 2 * iy + ((c >> 1) & 1)) * kMBX + 2 + 2 * ix + (c & 1); };
  // coarse plane of relative layer j (coarse cells (ox0 - 2, oy0 - 2) + [0, 20) x [0, 12) at z = oz0 + j)
  constexpr int kCPer = (kMCPlane + kMThreads - 1) / kMThreads;   // 2
  constexpr int kCR = PROLONG ? kCPer : 1;
  T cm2[kCR], cm1[kCR], cpf[kCR];   // coarse planes jw - 1, jw, jw + 1 of the layer jw written next
  auto coarse_load = [&](int j, T(&out)[kCR]) {
    const int lnc = lno - 1, mc = (1 << lnc) - 1;   // coarse grid: 2^lno cells, 2^(lno-1) octs per dimension
    const int Z = (oz0 + j) & ((1 << lno) - 1);
#pragma unroll
    for (int r = 0; r < kCR; ++r) {
      const int q = min(t + r * kMThreads, kMCPlane - 1);
      const int X = (ox0 - 2 + q % kMCX) & ((1 << lno) - 1), Y = (oy0 - 2 + q / kMCX) & ((1 << lno) - 1);
      const int64_t co = ((((int64_t)((Z >> 1) & mc) << lnc) + ((Y >> 1) & mc)) << lnc) + ((X >> 1) & mc);
      out[r] = ec[co * 8 + (X & 1) + 2 * (Y & 1) + 4 * (Z & 1)];
    }
  };
  if (PROLONG) {   // the planes of layer -1, and layer 0's upper one
    coarse_load(-2, cm2);
    coarse_load(-1, cm1);
    coarse_load(0, cpf);
  }

  auto step = [&](int st, auto G) {
    constexpr int g0 = decltype(G)::value;   // == st & 3
    // A: layer st - 1 into the ring (PROLONG: coarse plane st into its ring first)
    const int jw = st - 1;
    if (PROLONG && st >= 0 && st <= kz + 1) {
      // z-interpolated coarse planes of layer jw: cell plane 0 leans toward
      // coarse plane jw - 1, cell plane 1 toward jw + 1
#pragma unroll
      for (int r = 0; r < kCR; ++r) {
        const int q = t + r * kMThreads;
        if (q < kMCPlane) {
          zc[q] = T(0.75) * cm1[r] + T(0.25) * cm2[r];
          zc[kMCPlane + q] = T(0.75) * cm1[r] + T(0.25) * cpf[r];
        }
        cm2[r] = cm1[r];
        cm1[r] = cpf[r];
      }
      if (st + 1 <= kz + 1) coarse_load(st + 1, cpf);
      __syncthreads();
    }
    if (jw >= -1 && jw <= kz) {
      if (ZERO) {
        for (int q = t; q < 2 * kMPlane; q += kMThreads) s[plane_of(jw, q / kMPlane) * kMPlane + q % kMPlane] = T(0);
      } else {
#pragma unroll
        for (int r = 0; r < kPF; ++r) {
          const int q = t + r * kMThreads;
          if (q < kVec) {
            const int o = q / VPO, part = q % VPO;
            const int qx = o % kMBOX, qy = o / kMBOX;
            const T* pv = reinterpret_cast<const T*>(&pf[r]);
            T corr[VN];
            if (PROLONG) {
              // parent column (px, py) in the coarse plane; 3/4 parent + 1/4 neighbour per axis
              const T* Z = zc + ((part * VN) >> 2) * kMCPlane;
              const int px = 1 + qx, py = 1 + qy;
              if constexpr (VN == 2) {   // cells (0, cy) and (1, cy)
                const int yn = (part & 1) ? py + 1 : py - 1;
                T row[3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                  row[a] = T(0.75) * Z[py * kMCX + px - 1 + a] + T(0.25) * Z[yn * kMCX + px - 1 + a];
                corr[0] = T(0.75) * row[1] + T(0.25) * row[0];
                corr[1] = T(0.75) * row[1] + T(0.25) * row[2];
              } else {                   // cells (0, 0), (1, 0), (0, 1), (1, 1)
                T row[2][3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                  const T mid = Z[py * kMCX + px - 1 + a];
                  row[0][a] = T(0.75) * mid + T(0.25) * Z[(py - 1) * kMCX + px - 1 + a];
                  row[1][a] = T(0.75) * mid + T(0.25) * Z[(py + 1) * kMCX + px - 1 + a];
                }
#pragma unroll
                for (int cy = 0; cy < 2; ++cy) {
                  corr[2 * cy] = T(0.75) * row[cy][1] + T(0.25) * row[cy][0];
                  corr[2 * cy + 1] = T(0.75) * row[cy][1] + T(0.25) * row[cy][2];
                }
              }
            }
#pragma unroll
            for (int e = 0; e < VN; ++e) {
              const int c = part * VN + e;
              const int lx = 2 * qx + (c & 1), ly = 2 * qy + ((c >> 1) & 1);
              T val = pv[e];
              if (PROLONG) val += corr[e];
              s[plane_of(jw, c >> 2) * kMPlane + ly * kMBX + lx] = val;
            }
          }
        }
      }
    }
    // B: loads of layer st
    if (st >= -1 && st <= kz) {
      const int oz = (oz0 + st) & m;
      if (!ZERO) {
#pragma unroll
        for (int r = 0; r < kPF; ++r) {
          const int q = min(t + r * kMThreads, kVec - 1);
          const int o = q / VPO, part = q % VPO;
          const int qx = o % kMBOX, qy = o / kMBOX;
          pf[r] = reinterpret_cast<const V*>(phi + g.idx(ox0 - 1 + qx, oy0 - 1 + qy, oz) * 8)[part];
        }
      }
      const V* bv = reinterpret_cast<const V*>(b + g.idx(ox0 + ix, oy0 + iy, oz) * 8 + (8 - kMCPT) * hz);
#pragma unroll
      for (int k = 0; k < kMCPT / VN; ++k) {
        const V v = bv[k];
        const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
        for (int e = 0; e < VN; ++e) bo[g0][k * VN + e] = pv[e];
      }
      if (t < kMShell) {
        const int gx = 2 * ox0 - 2 + slx, gy = 2 * oy0 - 2 + sly;
        bs[g0] = b[g.idx(gx >> 1, gy >> 1, oz) * 8 + (gx & 1) + 2 * (gy & 1) + 4 * sp];
      }
    }
    __syncthreads();
    // C: norm of the incoming phi
    if (partials) {
      const int jl = st - 1, ju = st - 2;
#pragma unroll
      for (int j = 0; j < kMCPT; ++j) {
        const int c = cell(j), cz = c >> 2;
        const int jj = cz == 0 ? jl : ju;
        if (jj >= 0 && jj < kz) {
          const int P = plane_of(jj, cz), xy = own_xy(c);
          const T bv = cz == 0 ? bo[(g0 + 3) & 3][j] : bo[(g0 + 2) & 3][j];
          const T r = bv - (nsum(P, xy) - T(6) * s[P * kMPlane + xy]) * inv_h2;
          acc += (double)r * (double)r;
        }
      }
      __syncthreads();   // the red update below overwrites cells read above
    }
    // D: red update of layer st - 2 (column + one-cell xy ring)
    const int jr = st - 2;
    if (jr >= -1 && jr <= kz) {
#pragma unroll
      for (int j = 0; j < kMCPT; ++j) {
        const int c = cell(j), cz = c >> 2;
        if (colour_of(c) != 0) continue;
        if ((jr == -1 && cz == 0) || (jr == kz && cz == 1)) continue;
        const int P = plane_of(jr, cz), xy = own_xy(c);
        s[P * kMPlane + xy] = (nsum(P, xy) - h2 * bo[(g0 + 2) & 3][j]) * sixth;
      }
      if (t < kMShell && !((jr == -1 && sp == 0) || (jr == kz && sp == 1))) {
        const int P = plane_of(jr, sp), xy = sly * kMBX + slx;
        s[P * kMPlane + xy] = (nsum(P, xy) - h2 * bs[(g0 + 2) & 3]) * sixth;
      }
    }
    __syncthreads();
    // E: black update of layer st - 3, then store its octs
    const int jb = st - 3;
    if (jb >= 0 && jb < kz) {
      T out[kMCPT];
#pragma unroll
      for (int j = 0; j < kMCPT; ++j) {
        const int c = cell(j);
        const int P = plane_of(jb, c >> 2), xy = own_xy(c);
        out[j] = colour_of(c) == 0 ? s[P * kMPlane + xy] : (nsum(P, xy) - h2 * bo[(g0 + 1) & 3][j]) * sixth;
      }
      const int64_t first = g.idx(ox0 + ix, oy0 + iy, (oz0 + jb) & m) * 8 + (8 - kMCPT) * hz;   // own cells
      if (add64) {
        double2* av = reinterpret_cast<double2*>(add64 + first);
        double2 a[kMCPT / 2];
#pragma unroll
        for (int k = 0; k < kMCPT / 2; ++k) a[k] = av[k];
#pragma unroll
        for (int k = 0; k < kMCPT / 2; ++k) {
          a[k].x += (double)out[2 * k];
          a[k].y += (double)out[2 * k + 1];
          av[k] = a[k];
        }
      } else {
        V* dv = reinterpret_cast<V*>(dst + first);
#pragma unroll
        for (int k = 0; k < kMCPT / VN; ++k) {
          V v;
          T* pv = reinterpret_cast<T*>(&v);
#pragma unroll
          for (int e = 0; e < VN; ++e) pv[e] = out[k * VN + e];
          dv[k] = v;
        }
      }
    }
    __syncthreads();
  };
  // steps -1 .. kz + 2, four per iteration so that every ring slot index is a constant
  for (int s0 = -1; s0 < kz + 3; s0 += 4) {
    step(s0, std::integral_constant<int, 3>{});
    step(s0 + 1, std::integral_constant<int, 0>{});
    step(s0 + 2, std::integral_constant<int, 1>{});
    step(s0 + 3, std::integral_constant<int, 2>{});
  }
  if (partials) {
    const double tot = block_sum(acc);
    if (t == 0) partials[blockIdx.x] = tot;
  }
}

// ---- residual marching along z through an LDS ring ---------------------------
// The residual r = b - L phi on the column/run decomposition of the marching
// sweep (32 x 16-cell columns, runs of oct layers, XCD-ordered): phi of the
// column plus a one-oct halo streams through the same 8-plane ring, one oct
// layer per step (A: store layer st - 1 into the ring, B: issue the loads of
// layer st, C: residual of layer st - 2, whose two neighbouring layers are
// then in the ring).  phi is read about once (the x/y halo hits in L2), where
// the 3-D tile kernel re-reads its z halo.  MODE 0: the 8 residuals of each
// oct are averaged into its father cell on the grid n/2 (restriction);
// MODE 1: the norm only; MODE 2 (T = double): r rounded to FP32 per cell.
// With `partials`, one f64 ||r||^2 per workgroup.
template <typename T, int MODE>
__global__ __launch_bounds__(March<T>::threads) void k_resid_march(int lno, int chunks, T inv_h2,
                                                           const T* __restrict__ phi, const T* __restrict__ b,
                                                           T* __restrict__ bc, float* __restrict__ r32,
                                                           double* __restrict__ partials) {
  static_assert(MODE != 2 || sizeof(T) == 8, "the FP32 copy of the residual is made from FP64");
  constexpr int kMSplit = March<T>::split, kMCPT = March<T>::cpt, kMThreads = March<T>::threads;
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  constexpr int VPO = 8 / VN;
  constexpr int kVec = kMBOX * kMBOY * VPO;
  constexpr int kPF = (kVec + kMThreads - 1) / kMThreads;
  __shared__ T s[8 * kMPlane];
  __shared__ T rs[MODE == 0 && kMSplit == 2 ? kMOcts : 1];   // upper-plane sums of each oct (split threads)
  const int m = (1 << lno) - 1;
  const int n_cell = 2 << lno;
  const int ncx = n_cell / kMX, cols = ncx * (n_cell / kMY);
  const int nb = cols * chunks;
  int u = blockIdx.x;
  if ((nb & 7) == 0) u = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int col = u % cols, chunk = u / cols;
  const int ox0 = (col % ncx) * kMOX, oy0 = (col / ncx) * kMOY;
  const int oz0 = (chunk << lno) / chunks;
  const int kz = ((chunk + 1) << lno) / chunks - oz0;
  const OctGeom g{lno, m};
  const int t = threadIdx.x;
  const int to = t % kMOcts, hz = kMSplit == 1 ? 0 : t / kMOcts;
  const int ix = to % kMOX, iy = to / kMOX;
  auto cell = [&](int j) { return kMSplit == 1 ? j : 4 * hz + j; };
  auto plane_of = [](int j, int cz) { return (2 * j + cz + 8) & 7; };
  auto own_xy = [&](int c) { return (2 + 2 * iy + ((c >> 1) & 1)) * kMBX + 2 + 2 * ix + (c & 1); };
  V pf[kPF];
  T bo[4][kMCPT];   // b of the own cells, layer j in slot j & 3
  double acc = 0.0;

  auto step = [&](int st, auto G) {
    constexpr int g0 = decltype(G)::value;   // == st & 3
    // A: layer st - 1 into the ring
    const int jw = st - 1;
    if (jw >= -1 && jw <= kz) {
#pragma unroll
      for (int r = 0; r < kPF; ++r) {
        const int q = t + r * kMThreads;
        if (q < kVec) {
          const int o = q / VPO, part = q % VPO;
          const int qx = o % kMBOX, qy = o / kMBOX;
          const T* pv = reinterpret_cast<const T*>(&pf[r]);
#pragma unroll
          for (int e = 0; e < VN; ++e) {
            const int c = part * VN + e;
            s[plane_of(jw, c >> 2) * kMPlane + (2 * qy + ((c >> 1) & 1)) * kMBX + 2 * qx + (c & 1)] = pv[e];
          }
        }
      }
    }
    // B: loads of layer st (phi box; b of the own cells for the layers of the run)
    if (st >= -1 && st <= kz) {
      const int oz = (oz0 + st) & m;
#pragma unroll
      for (int r = 0; r < kPF; ++r) {
        const int q = min(t + r * kMThreads, kVec - 1);
        const int o = q / VPO, part = q % VPO;
        const int qx = o % kMBOX, qy = o / kMBOX;
        pf[r] = reinterpret_cast<const V*>(phi + g.idx(ox0 - 1 + qx, oy0 - 1 + qy, oz) * 8)[part];
      }
      if (st >= 0 && st < kz) {
        const V* bv = reinterpret_cast<const V*>(b + g.idx(ox0 + ix, oy0 + iy, oz) * 8 + (8 - kMCPT) * hz);
#pragma unroll
        for (int k = 0; k < kMCPT / VN; ++k) {
          const V v = bv[k];
          const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
          for (int e = 0; e < VN; ++e) bo[g0][k * VN + e] = pv[e];
        }
      }
    }
    __syncthreads();
    // C: residual of layer st - 2 (layers st - 3 and st - 1 are in the ring)
    const int jr = st - 2;
    if (jr >= 0 && jr < kz) {
      T rsum = T(0);
      float rf[kMCPT];
#pragma unroll
      for (int j = 0; j < kMCPT; ++j) {
        const int c = cell(j);
        const int i = plane_of(jr, c >> 2) * kMPlane + own_xy(c);
        const T sum = s[i - 1] + s[i + 1] + s[i - kMBX] + s[i + kMBX] + s[((plane_of(jr, c >> 2) + 7) & 7) * kMPlane + own_xy(c)] +
                      s[((plane_of(jr, c >> 2) + 1) & 7) * kMPlane + own_xy(c)];
        const T r = bo[(g0 + 2) & 3][j] - (sum - T(6) * s[i]) * inv_h2;
        rsum += r;
        rf[j] = (float)r;
        acc += (double)r * (double)r;
      }
      const int oz = (oz0 + jr) & m;
      if (MODE == 2) {
        float4* rv = reinterpret_cast<float4*>(r32 + g.idx(ox0 + ix, oy0 + iy, oz) * 8 + (8 - kMCPT) * hz);
#pragma unroll
        for (int k = 0; k < kMCPT / 4; ++k) rv[k] = float4{rf[4 * k], rf[4 * k + 1], rf[4 * k + 2], rf[4 * k + 3]};
      }
      if (MODE == 0) {
        if (kMSplit == 2 && hz == 1) rs[to] = rsum;
        if (kMSplit == 2) __syncthreads();
        if (hz == 0) {
          if (kMSplit == 2) rsum += rs[to];
          const int ox = ox0 + ix, oy = oy0 + iy;   // the father cell on the grid n/2
          const int lnc = lno - 1;
          const int64_t co = ((((int64_t)(oz >> 1) << lnc) + (oy >> 1)) << lnc) + (ox >> 1);
          bc[co * 8 + (ox & 1) + 2 * (oy & 1) + 4 * (oz & 1)] = rsum * T(0.125);
        }
      }
    }
    __syncthreads();
  };
  // steps -1 .. kz + 1, four per iteration so that every ring slot index is a constant
  for (int s0 = -1; s0 < kz + 2; s0 += 4) {
    step(s0, std::integral_constant<int, 3>{});
    step(s0 + 1, std::integral_constant<int, 0>{});
    step(s0 + 2, std::integral_constant<int, 1>{});
    step(s0 + 3, std::integral_constant<int, 2>{});
  }
  if (partials) {
    const double tot = block_sum(acc);
    if (t == 0) partials[blockIdx.x] = tot;
  }
}

// ---- outer residual of the mixed solve fused with the first FP32 sweep ----------
// Each outer step of the FP32-in-FP64 solve forms r = f - L phi in FP64,
// rounds it to FP32 (RNE) as the right-hand side of an FP32 V-cycle from a
// zero guess, whose first red-black sweep is then a local stencil of r:
// red cells e = (0 - h^2 r) / 6, black cells e = (sum of the six red e -
// h^2 r) / 6.  Both are done in one pass: phi (FP64) streams through an
// 8-plane ring of the column + one-oct halo; step s stores layer s-1, loads
// layer s, forms r on layer s-2 for the column and its one-cell xy ring (red
// cells keep their e, black cells their r, in a second, FP32 ring), stores
// r32 and the FP64 norm partial of the column; and takes the black update of
// layer s-3, whose red neighbours are then in the FP32 ring, storing e of
// the column.  The FP32 arithmetic is that of the zero-guess sweep.
constexpr int kOShell = ((kMX + 2) * (kMY + 2) - kMX * kMY) * 2;   // 1-ring cells of one oct layer: 200
struct OuterShell {
  uint16_t v[kOShell];   // lx | ly << 6 | plane << 12
};
constexpr OuterShell make_outer_shell() {
  OuterShell t{};
  int k = 0;
  for (int p = 0; p < 2; ++p)
    for (int y = 1; y < kMBY - 1; ++y)
      for (int x = 1; x < kMBX - 1; ++x) {
        const bool inner = x >= 2 && x < kMBX - 2 && y >= 2 && y < kMBY - 2;
        if (!inner) t.v[k++] = (uint16_t)(x | (y << 6) | (p << 12));
      }
  return t;
}
__constant__ OuterShell kOuterShell = make_outer_shell();
static_assert(kOShell <= 256, "one ring cell per thread");
__global__ __launch_bounds__(256) void k_outer_resid_sweep(int lno, int chunks, double inv_h2, float h2f,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ f, float* __restrict__ r32,
                                                           float* __restrict__ e32, double* __restrict__ partials) {
  constexpr int kThreads = 256, kCPT = 4;
  constexpr int VPO = 4;                                      // double2 pieces per oct
  constexpr int kVec = kMBOX * kMBOY * VPO;
  constexpr int kPF = (kVec + kThreads - 1) / kThreads;
  __shared__ double s[8 * kMPlane];       // phi ring (FP64)
  __shared__ float se[8 * kMPlane];       // red: e, black: r32 (FP32 ring)
  const int m = (1 << lno) - 1;
  const int n_cell = 2 << lno;
  const int ncx = n_cell / kMX, cols = ncx * (n_cell / kMY);
  const int nb = cols * chunks;
  int u = blockIdx.x;
  if ((nb & 7) == 0) u = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int col = u % cols, chunk = u / cols;
  const int ox0 = (col % ncx) * kMOX, oy0 = (col / ncx) * kMOY;
  const int oz0 = (chunk << lno) / chunks;
  const int kz = ((chunk + 1) << lno) / chunks - oz0;
  const OctGeom g{lno, m};
  const int t = threadIdx.x;
  const int to = t % kMOcts, hz = t / kMOcts;
  const int ix = to % kMOX, iy = to / kMOX;
  // this thread's ring cell (one-cell xy ring of the column, both planes)
  int glx = 0, gly = 0, gp = 0;
  if (t < kOShell) {
    const int v = kOuterShell.v[t];
    glx = v & 63;
    gly = (v >> 6) & 63;
    gp = v >> 12;
  }
  const float sixth = 1.0f / 6.0f;
  double2 pf[kPF];
  double fo[4][kCPT];   // f of the own cells, layer j in slot j & 3
  double fs[4];         // f of the ring cell
  double acc = 0.0;
  auto plane_of = [](int j, int cz) { return (2 * j + cz + 8) & 7; };
  auto own_xy = [&](int c) { return (2 + 2 * iy + ((c >> 1) & 1)) * kMBX + 2 + 2 * ix + (c & 1); };
  auto nsum64 = [&](int P, int xy) {
    const int i = P * kMPlane + xy;
    return s[i - 1] + s[i + 1] + s[i - kMBX] + s[i + kMBX] + s[((P + 7) & 7) * kMPlane + xy] +
           s[((P + 1) & 7) * kMPlane + xy];
  };
  auto nsum32 = [&](int P, int xy) {
    const int i = P * kMPlane + xy;
    return se[i - 1] + se[i + 1] + se[i - kMBX] + se[i + kMBX] + se[((P + 7) & 7) * kMPlane + xy] +
           se[((P + 1) & 7) * kMPlane + xy];
  };
  // residual of one cell (FP64), rounded to FP32; the FP32 ring gets e (red) or r32 (black)
  auto resid_cell = [&](int P, int xy, double fv, bool red) {
    const double r = fv - (nsum64(P, xy) - 6.0 * s[P * kMPlane + xy]) * inv_h2;
    const float rf = (float)r;
    se[P * kMPlane + xy] = red ? (0.0f - h2f * rf) * sixth : rf;
    return r;
  };

  auto step = [&](int st, auto G) {
    constexpr int g0 = decltype(G)::value;   // == st & 3
    // A: layer st - 1 into the FP64 ring
    const int jw = st - 1;
    if (jw >= -1 && jw <= kz) {
#pragma unroll
      for (int r = 0; r < kPF; ++r) {
        const int q = t + r * kThreads;
        if (q < kVec) {
          const int o = q / VPO, part = q % VPO;
          const int qx = o % kMBOX, qy = o / kMBOX;
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int c = part * 2 + e;
            s[plane_of(jw, c >> 2) * kMPlane + (2 * qy + ((c >> 1) & 1)) * kMBX + 2 * qx + (c & 1)] =
                e == 0 ? pf[r].x : pf[r].y;
          }
        }
      }
    }
    // B: loads of layer st
    if (st >= -1 && st <= kz) {
      const int oz = (oz0 + st) & m;
#pragma unroll
      for (int r = 0; r < kPF; ++r) {
        const int q = min(t + r * kThreads, kVec - 1);
        const int o = q / VPO, part = q % VPO;
        const int qx = o % kMBOX, qy = o / kMBOX;
        pf[r] = reinterpret_cast<const double2*>(phi + g.idx(ox0 - 1 + qx, oy0 - 1 + qy, oz) * 8)[part];
      }
      const double2* fv = reinterpret_cast<const double2*>(f + g.idx(ox0 + ix, oy0 + iy, oz) * 8 + 4 * hz);
      const double2 a = fv[0], bq = fv[1];
      fo[g0][0] = a.x;
      fo[g0][1] = a.y;
      fo[g0][2] = bq.x;
      fo[g0][3] = bq.y;
      if (t < kOShell) {
        const int gx = 2 * ox0 - 2 + glx, gy = 2 * oy0 - 2 + gly;
        fs[g0] = f[g.idx(gx >> 1, gy >> 1, oz) * 8 + (gx & 1) + 2 * (gy & 1) + 4 * gp];
      }
    }
    __syncthreads();
    // R: residual of layer st - 2 on the column (stored, summed) and its one-cell ring
    const int jr = st - 2;
    if (jr >= -1 && jr <= kz) {
      const bool own_layer = jr >= 0 && jr < kz;
      if (own_layer) {
        float rf[kCPT];
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
          const int c = 4 * hz + j;
          const double r = resid_cell(plane_of(jr, hz), own_xy(c), fo[(g0 + 2) & 3][j], colour_of(c) == 0);
          rf[j] = (float)r;
          acc += r * r;
        }
        *reinterpret_cast<float4*>(r32 + g.idx(ox0 + ix, oy0 + iy, (oz0 + jr) & m) * 8 + 4 * hz) =
            float4{rf[0], rf[1], rf[2], rf[3]};
      }
      // the ring cells of the run's own layers
      if (t < kOShell && own_layer) {
        const bool red = ((glx + gly + gp) & 1) == 0;
        resid_cell(plane_of(jr, gp), gly * kMBX + glx, fs[(g0 + 2) & 3], red);
      }
      // the column cells of the z halo planes next to the run
      if (!own_layer && ((jr == -1 && hz == 1) || (jr == kz && hz == 0))) {
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
          const int c = 4 * hz + j;
          resid_cell(plane_of(jr, hz), own_xy(c), fo[(g0 + 2) & 3][j], colour_of(c) == 0);
        }
      }
    }
    __syncthreads();
    // E: black update of layer st - 3 (the column), store e
    const int jb = st - 3;
    if (jb >= 0 && jb < kz) {
      float out[kCPT];
#pragma unroll
      for (int j = 0; j < kCPT; ++j) {
        const int c = 4 * hz + j;
        const int P = plane_of(jb, hz), xy = own_xy(c);
        out[j] = colour_of(c) == 0 ? se[P * kMPlane + xy] : (nsum32(P, xy) - h2f * se[P * kMPlane + xy]) * sixth;
      }
      *reinterpret_cast<float4*>(e32 + g.idx(ox0 + ix, oy0 + iy, (oz0 + jb) & m) * 8 + 4 * hz) =
          float4{out[0], out[1], out[2], out[3]};
    }
    __syncthreads();
  };
  for (int s0 = -1; s0 < kz + 3; s0 += 4) {
    step(s0, std::integral_constant<int, 3>{});
    step(s0 + 1, std::integral_constant<int, 0>{});
    step(s0 + 2, std::integral_constant<int, 1>{});
    step(s0 + 3, std::integral_constant<int, 2>{});
  }
  const double tot = block_sum(acc);
  if (t == 0) partials[blockIdx.x] = tot;
}

// ---- residual on an LDS tile --------------------------------------------------
// One workgroup per 16 x 16 x 8 tile stages phi with a one-oct halo (as the
// sweep does) and forms r = b - L phi for its own octs, one oct per thread.
// MODE 0: the oct's 8 residuals are averaged into the father cell on the grid
// n/2 (restriction); MODE 1: nothing but the norm; MODE 2 (T = double, the
// outer loop of the mixed solve): r rounded to FP32 per cell into r32; MODE 3
// (T = double): b is not given but formed on the fly as bscale (rho - *bmean)
// from the density passed as `b`, and ||b||^2 goes to partials_b as well.
// With `partials`, one f64 ||r||^2 per tile.
template <typename T, int MODE>
__global__ __launch_bounds__(kTileThreads) void k_resid_tile(int lno, T inv_h2, const T* __restrict__ phi,
                                                             const T* __restrict__ b, T* __restrict__ bc,
                                                             float* __restrict__ r32, double* __restrict__ partials,
                                                             double bscale, const double* __restrict__ bmean,
                                                             double* __restrict__ partials_b) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  constexpr int VPO = 8 / VN;
  __shared__ T s[kLX * kLY * kLZ];
  const int n_cell = 2 << lno;
  const int m = (1 << lno) - 1;
  const int tnx = n_cell / kTX, tny = n_cell / kTY, tnz = n_cell / kTZ;
  const int nb = tnx * tny * tnz;
  int tile = blockIdx.x;
  if ((nb & 7) == 0) tile = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int tx = tile % tnx, ty = (tile / tnx) % tny, tz = tile / (tnx * tny);
  const int ox0 = tx * (kTX / 2), oy0 = ty * (kTY / 2), oz0 = tz * (kTZ / 2);
  const OctGeom g{lno, m};
  const int t = threadIdx.x;
  const int ix = t % (kTX / 2), iy = (t / (kTX / 2)) % (kTY / 2), iz = t / ((kTX / 2) * (kTY / 2));
  const int64_t my_oct = g.idx(ox0 + ix, oy0 + iy, oz0 + iz);
  T bo[8];
  {
    const V* bv = reinterpret_cast<const V*>(b + my_oct * 8);
#pragma unroll
    for (int k = 0; k < VPO; ++k) {
      const V v = bv[k];
      const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
      for (int j = 0; j < VN; ++j) bo[k * VN + j] = pv[j];
    }
  }
  double accb = 0.0;
  if (MODE == 3) {
    const double mu = bmean[0];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      bo[c] = (T)(bscale * ((double)bo[c] - mu));
      accb += (double)bo[c] * (double)bo[c];
    }
  }
  constexpr int kStageVec = kRX * kRY * kRZ * VPO;
  constexpr int kStagePer = (kStageVec + kTileThreads - 1) / kTileThreads;
  V sv[kStagePer];
#pragma unroll
  for (int r = 0; r < kStagePer; ++r) {
    const int q = min(t + r * kTileThreads, kStageVec - 1);
    const int o = q / VPO, part = q % VPO;
    const int qx = o % kRX, qy = (o / kRX) % kRY, qz = o / (kRX * kRY);
    sv[r] = reinterpret_cast<const V*>(phi + g.idx(ox0 - 1 + qx, oy0 - 1 + qy, oz0 - 1 + qz) * 8)[part];
  }
#pragma unroll
  for (int r = 0; r < kStagePer; ++r) {
    const int q = t + r * kTileThreads;
    if (q < kStageVec) {
      const int o = q / VPO, part = q % VPO;
      const int qx = o % kRX, qy = (o / kRX) % kRY, qz = o / (kRX * kRY);
      const T* pv = reinterpret_cast<const T*>(&sv[r]);
#pragma unroll
      for (int j = 0; j < VN; ++j) {
        const int c = part * VN + j;
        s[lds_idx(2 * qx + (c & 1), 2 * qy + ((c >> 1) & 1), 2 * qz + (c >> 2))] = pv[j];
      }
    }
  }
  __syncthreads();
  const int i0 = lds_idx(2 * ix + 2, 2 * iy + 2, 2 * iz + 2);
  double acc = 0.0;
  T rsum = T(0);
  float rf[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int i = i0 + (c & 1) + ((c >> 1) & 1) * kLX + (c >> 2) * kLX * kLY;
    const T sum = s[i - 1] + s[i + 1] + s[i - kLX] + s[i + kLX] + s[i - kLX * kLY] + s[i + kLX * kLY];
    const T r = bo[c] - (sum - T(6) * s[i]) * inv_h2;
    rsum += r;
    rf[c] = (float)r;
    acc += (double)r * (double)r;
  }
  if (MODE == 0) {
    const int ox = ox0 + ix, oy = oy0 + iy, oz = oz0 + iz;   // = the father cell on the grid n/2
    const int lnc = lno - 1;
    const int64_t co = ((((int64_t)(oz >> 1) << lnc) + (oy >> 1)) << lnc) + (ox >> 1);
    bc[co * 8 + (ox & 1) + 2 * (oy & 1) + 4 * (oz & 1)] = rsum * T(0.125);
  } else if (MODE == 2) {
    float4* rv = reinterpret_cast<float4*>(r32 + my_oct * 8);
    rv[0] = float4{rf[0], rf[1], rf[2], rf[3]};
    rv[1] = float4{rf[4], rf[5], rf[6], rf[7]};
  }
  if (partials) {
    const double tot = block_sum(acc);
    if (t == 0) partials[blockIdx.x] = tot;
  }
  if (MODE == 3) {
    __syncthreads();   // block_sum's shared slots are reused
    const double totb = block_sum(accb);
    if (t == 0) partials_b[blockIdx.x] = totb;
  }
}

// ---- the whole V-cycle below 16^3 in one workgroup ----------------------------
// Levels n0 (16 or 8), n0/2, ..., 4 live in LDS as dense grids (x fastest):
// zero guess, nu_pre red-black sweeps, residual + 8-child restriction down to
// 4^3, pseudo-inverse solve there, trilinear prolongation + nu_post sweeps on
// the way up.  The same arithmetic as the per-level kernels, without ~25
// kernel launches per cycle.
constexpr int kSmallMax = 16 * 16 * 16 + 8 * 8 * 8 + 4 * 4 * 4;

// one colour of a red-black sweep on a dense periodic n^3 grid in LDS
// (n = 2^lg): the thread enumerates only cells of that colour
template <typename T>
__device__ __forceinline__ void small_smooth(T* e, const T* b, int lg, T h2, int colour) {
  const int n = 1 << lg, m = n - 1;
  const int half = 1 << (3 * lg - 1);
  const T sixth = T(1) / T(6);
  for (int k = threadIdx.x; k < half; k += blockDim.x) {
    const int y = (k >> (lg - 1)) & m, z = k >> (2 * lg - 1);
    const int x = 2 * (k & ((n >> 1) - 1)) + ((y + z + colour) & 1);
    const int i = (z * n + y) * n + x;
    const T sn = e[(z * n + y) * n + ((x - 1) & m)] + e[(z * n + y) * n + ((x + 1) & m)] +
                 e[(z * n + ((y - 1) & m)) * n + x] + e[(z * n + ((y + 1) & m)) * n + x] +
                 e[(((z - 1) & m) * n + y) * n + x] + e[(((z + 1) & m) * n + y) * n + x];
    e[i] = (sn - h2 * b[i]) * sixth;
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_vcycle_small(int n0, T h0, const T* __restrict__ bg, T* __restrict__ eg,
                                                       const T* __restrict__ G, int nu_pre, int nu_post) {
  __shared__ T se[kSmallMax];
  __shared__ T sb[kSmallMax];
  int nl = 0, off[3], nn[3];
  for (int n = n0, o = 0; n >= 4; n >>= 1, ++nl) {
    off[nl] = o;
    nn[nl] = n;
    o += n * n * n;
  }
  const int lno0 = __ffs(n0) - 2;              // log2(n0 / 2)
  auto octidx = [](int x, int y, int z, int lno) {
    return ((((z >> 1) << lno) + (y >> 1)) << lno) + (x >> 1);
  };
  // the 4^3 pseudo-inverse, fetched now for use at the bottom of the cycle:
  // thread t holds G[cell t / 16][cells 4 (t % 16) .. + 3] (oct-major order)
  const int gi = threadIdx.x >> 4, gj0 = (threadIdx.x & 15) * 4;
  T greg[4];
  {
    const int x = gi & 3, y = (gi >> 2) & 3, z = gi >> 4;
    const int qi = octidx(x, y, z, 1) * 8 + (x & 1) + 2 * (y & 1) + 4 * (z & 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = gj0 + k, xj = j & 3, yj = (j >> 2) & 3, zj = j >> 4;
      const int qj = octidx(xj, yj, zj, 1) * 8 + (xj & 1) + 2 * (yj & 1) + 4 * (zj & 1);
      greg[k] = G[qi * 64 + qj];
    }
  }
  const int lg0 = lno0 + 1;                     // log2(n0)
  for (int i = threadIdx.x; i < n0 * n0 * n0; i += blockDim.x) {
    const int x = i & (n0 - 1), y = (i >> lg0) & (n0 - 1), z = i >> (2 * lg0);
    sb[i] = bg[octidx(x, y, z, lno0) * 8 + (x & 1) + 2 * (y & 1) + 4 * (z & 1)];
    se[i] = T(0);
  }
  __syncthreads();
  // down: smooth, residual + restriction
  for (int l = 0; l + 1 < nl; ++l) {
    const int n = nn[l], m = n - 1;
    const T h = h0 * T(n0 / n), h2 = h * h, inv_h2 = T(1) / h2;
    T* e = se + off[l];
    const T* b = sb + off[l];
    const int lg = lg0 - l;
    for (int it = 0; it < nu_pre; ++it) {
      small_smooth(e, b, lg, h2, 0);
      __syncthreads();
      small_smooth(e, b, lg, h2, 1);
      __syncthreads();
    }
    const int nc = n / 2, Nc = nc * nc * nc;
    for (int I = threadIdx.x; I < Nc; I += blockDim.x) {
      const int X = I % nc, Y = (I / nc) % nc, Z = I / (nc * nc);
      T rsum = T(0);
      for (int c = 0; c < 8; ++c) {
        const int x = 2 * X + (c & 1), y = 2 * Y + ((c >> 1) & 1), z = 2 * Z + (c >> 2);
        const T sn = e[(z * n + y) * n + ((x - 1) & m)] + e[(z * n + y) * n + ((x + 1) & m)] +
                     e[(z * n + ((y - 1) & m)) * n + x] + e[(z * n + ((y + 1) & m)) * n + x] +
                     e[(((z - 1) & m) * n + y) * n + x] + e[(((z + 1) & m) * n + y) * n + x];
        rsum += b[(z * n + y) * n + x] - (sn - T(6) * e[(z * n + y) * n + x]) * inv_h2;
      }
      sb[off[l + 1] + I] = rsum * T(0.125);
      se[off[l + 1] + I] = T(0);
    }
    __syncthreads();
  }
  // coarsest 4^3: e = G b, 16 threads per output cell, 4 products each,
  // summed across the 16-lane group in a fixed order
  {
    T* e = se + off[nl - 1];
    const T* b = sb + off[nl - 1];
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc += greg[k] * b[gj0 + k];
    for (int sh = 8; sh > 0; sh >>= 1) acc += __shfl_xor(acc, sh, 64);
    if ((threadIdx.x & 15) == 0) e[gi] = acc;
    __syncthreads();
  }
  // up: prolongation + correction, smooth
  for (int l = nl - 2; l >= 0; --l) {
    const int n = nn[l], nc = n / 2, mc = nc - 1;
    const T h = h0 * T(n0 / n), h2 = h * h;
    T* e = se + off[l];
    const T* ec = se + off[l + 1];
    const T w[2] = {T(0.75), T(0.25)};
    for (int i = threadIdx.x; i < n * n * n; i += blockDim.x) {
      const int x = i % n, y = (i / n) % n, z = i / (n * n);
      const int X = x >> 1, Y = y >> 1, Z = z >> 1;
      const int sx = (x & 1) ? 1 : -1, sy = (y & 1) ? 1 : -1, sz = (z & 1) ? 1 : -1;
      T v = T(0);
      for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb)
          for (int cc = 0; cc < 2; ++cc)
            v += (w[a] * w[bb] * w[cc]) *
                 ec[(((Z + cc * sz) & mc) * nc + ((Y + bb * sy) & mc)) * nc + ((X + a * sx) & mc)];
      e[i] += v;
    }
    __syncthreads();
    for (int it = 0; it < nu_post; ++it) {
      small_smooth(e, sb + off[l], lg0 - l, h2, 0);
      __syncthreads();
      small_smooth(e, sb + off[l], lg0 - l, h2, 1);
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n0 * n0 * n0; i += blockDim.x) {
    const int x = i & (n0 - 1), y = (i >> lg0) & (n0 - 1), z = i >> (2 * lg0);
    eg[octidx(x, y, z, lno0) * 8 + (x & 1) + 2 * (y & 1) + 4 * (z & 1)] = se[i];
  }
}

// ---- residual (+ restriction to the father cell) + f64 norm partials ------
template <typename T, bool RESTRICT>
__global__ __launch_bounds__(kBlock) void k_resid(int lno, T inv_h2, const T* __restrict__ phi,
                                                  const T* __restrict__ b, T* __restrict__ bc,
                                                  double* __restrict__ partials) {
  const int64_t n_oct = (int64_t)1 << (3 * lno);
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (o < n_oct) {
    const OctGeom g{lno, (1 << lno) - 1};
    int ox, oy, oz;
    oct_coords(o, lno, g.m, ox, oy, oz);
    const int64_t nb[6] = {g.idx(ox - 1, oy, oz), g.idx(ox + 1, oy, oz), g.idx(ox, oy - 1, oz),
                           g.idx(ox, oy + 1, oz), g.idx(ox, oy, oz - 1), g.idx(ox, oy, oz + 1)};
    T own[8], bo[8];
    load8(phi + o * 8, own);
    load8(b + o * 8, bo);
    T rsum = T(0);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const T s = nbr_sum(phi, own, nb, c);
      const T r = bo[c] - (s - T(6) * own[c]) * inv_h2;
      rsum += r;
      acc += (double)r * (double)r;
    }
    if (RESTRICT) {
      // father cell (ox, oy, oz) on the coarse grid of 2^lno cells per dimension
      const int lnc = lno - 1;
      const int64_t co = ((((int64_t)(oz >> 1) << lnc) + (oy >> 1)) << lnc) + (ox >> 1);
      bc[co * 8 + (ox & 1) + 2 * (oy & 1) + 4 * (oz & 1)] = rsum * T(0.125);
    }
  }
  if (partials) {
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

// ---- prolongation + correction -------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(int lno, const T* __restrict__ ec, T* __restrict__ e) {
  const int64_t n_oct = (int64_t)1 << (3 * lno);
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_oct) return;
  const int m = (1 << lno) - 1;   // coarse cells per dimension - 1
  const int lnc = lno - 1;        // log2(coarse octs per dimension)
  int X, Y, Z;
  oct_coords(o, lno, m, X, Y, Z);  // father coarse cell
  T E[3][3][3];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = (X + dx) & m, y = (Y + dy) & m, z = (Z + dz) & m;
        const int64_t co = ((((int64_t)(z >> 1) << lnc) + (y >> 1)) << lnc) + (x >> 1);
        E[dz + 1][dy + 1][dx + 1] = ec[co * 8 + (x & 1) + 2 * (y & 1) + 4 * (z & 1)];
      }
  const T w[2] = {T(0.75), T(0.25)};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int sx = (c & 1) ? 1 : -1, sy = (c & 2) ? 1 : -1, sz = (c & 4) ? 1 : -1;
    T v = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
          v += (w[a] * w[bb] * w[cc]) * E[1 + cc * sz][1 + bb * sy][1 + a * sx];
    e[o * 8 + c] += v;
  }
}

// ---- dense <-> oct-major layout of a periodic field (f64) --------------------
// Dense: (x n + y) n + z, z fastest.  Oct-major: oct (oz no + oy) no + ox,
// cell cx + 2 cy + 4 cz.  A workgroup moves a 32 x 2 x 32-cell tile (x, y, z)
// through LDS: on the dense side 64 runs of 32 consecutive z values (256 B),
// on the oct side 16 runs of 16 consecutive octs (1 KB: one oct layer in z of
// one oct row in y), so both sides are read and written in whole lines.
constexpr int kLT = 32;
constexpr int kLTP = kLT + 1;   // padded z row of the LDS tile
template <bool TO_OCT>
__global__ __launch_bounds__(256) void k_layout_tiled(int lg, const double* __restrict__ in,
                                                      double* __restrict__ out) {
  __shared__ double st[kLT * 2 * kLTP];   // [x][y][z]
  const int n = 1 << lg, no = n >> 1, tx = n / kLT;
  const int b = (int)blockIdx.x;
  const int xt = b % tx, yo = (b / tx) % no, zt = b / (tx * no);
  const int x0 = xt * kLT, y0 = 2 * yo, z0 = zt * kLT, xo0 = x0 >> 1, zo0 = z0 >> 1;
  constexpr int kPer = kLT * 2 * kLT / 256;   // 8 cells per thread
  if (TO_OCT) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int d = (int)threadIdx.x + 256 * k, zl = d & (kLT - 1), yl = (d >> 5) & 1, xl = d >> 6;
      st[(xl * 2 + yl) * kLTP + zl] = in[((int64_t)(x0 + xl) * n + y0 + yl) * n + z0 + zl];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = (int)threadIdx.x + 256 * k, row = e >> 7, w = e & 127, c = w & 7;
      const int xl = 2 * (w >> 3) + (c & 1), yl = (c >> 1) & 1, zl = 2 * row + (c >> 2);
      out[(((int64_t)(zo0 + row) * no + yo) * no + xo0 + (w >> 3)) * 8 + c] = st[(xl * 2 + yl) * kLTP + zl];
    }
  } else {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = (int)threadIdx.x + 256 * k, row = e >> 7, w = e & 127, c = w & 7;
      const int xl = 2 * (w >> 3) + (c & 1), yl = (c >> 1) & 1, zl = 2 * row + (c >> 2);
      st[(xl * 2 + yl) * kLTP + zl] = in[(((int64_t)(zo0 + row) * no + yo) * no + xo0 + (w >> 3)) * 8 + c];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int d = (int)threadIdx.x + 256 * k, zl = d & (kLT - 1), yl = (d >> 5) & 1, xl = d >> 6;
      out[((int64_t)(x0 + xl) * n + y0 + yl) * n + z0 + zl] = st[(xl * 2 + yl) * kLTP + zl];
    }
  }
}

// grids narrower than a tile: one thread per cell, indexed on the oct side
template <bool TO_OCT>
__global__ __launch_bounds__(kBlock) void k_layout_small(int lg, const double* __restrict__ in,
                                                         double* __restrict__ out) {
  const int n = 1 << lg, no = n >> 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * n * n) return;
  const int c = (int)(i & 7);
  const int64_t o = i >> 3;
  const int ox = (int)(o % no), oy = (int)((o / no) % no), oz = (int)(o / ((int64_t)no * no));
  const int x = 2 * ox + (c & 1), y = 2 * oy + ((c >> 1) & 1), z = 2 * oz + (c >> 2);
  const int64_t d = ((int64_t)x * n + y) * n + z;
  if (TO_OCT) out[i] = in[d];
  else out[d] = in[i];
}

// ---- coarsest grid: dense pseudo-inverse matvec, one workgroup -------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse(int N, const T* __restrict__ G, const T* __restrict__ b,
                                                   T* __restrict__ e) {
  __shared__ T bs[512];   // up to 8^3 coarsest cells
  for (int j = threadIdx.x; j < N; j += blockDim.x) bs[j] = b[j];
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    T acc = T(0);
    for (int j = 0; j < N; ++j) acc += G[(int64_t)i * N + j] * bs[j];
    e[i] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill_zero(T* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

// f = c (rho - mean) and per-workgroup partial sums of f^2: each thread takes
// kRhsPer elements kBlock apart (loads all issued first; indices past n load
// element n - 1, are not stored and count 0), summed in a fixed order.
constexpr int kRhsPer = 8;
__global__ __launch_bounds__(kBlock) void k_rhs(int64_t n, const double* __restrict__ rho,
                                                const double* __restrict__ d_mean, double c,
                                                double* __restrict__ f, double* __restrict__ partials) {
  const int64_t base = (int64_t)blockIdx.x * (kBlock * kRhsPer) + threadIdx.x;
  double v[kRhsPer];
#pragma unroll
  for (int j = 0; j < kRhsPer; ++j) v[j] = rho[min(base + (int64_t)j * kBlock, n - 1)];
  const double mean = d_mean[0];
#pragma unroll
  for (int j = 0; j < kRhsPer; ++j) {
    const int64_t i = base + (int64_t)j * kBlock;
    v[j] = c * (v[j] - mean);
    if (i < n) {
      if (f) f[i] = v[j];
    } else {
      v[j] = 0.0;
    }
  }
  const double a = ((v[0] * v[0] + v[1] * v[1]) + (v[2] * v[2] + v[3] * v[3])) +
                   ((v[4] * v[4] + v[5] * v[5]) + (v[6] * v[6] + v[7] * v[7]));
  const double t = block_sum(a);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Per-workgroup partial sums of x (reduced by k_reduce_final): each thread
// adds kSumPer elements kBlock apart (coalesced loads, all issued before the
// first add; indices past n load element n - 1 and count 0) in a fixed order.
constexpr int kSumPer = 8;
__global__ __launch_bounds__(kBlock) void k_partial_sum(int64_t n, const double* __restrict__ x,
                                                        double* __restrict__ partials) {
  const int64_t base = (int64_t)blockIdx.x * (kBlock * kSumPer) + threadIdx.x;
  double v[kSumPer];
#pragma unroll
  for (int j = 0; j < kSumPer; ++j) v[j] = x[min(base + (int64_t)j * kBlock, n - 1)];
#pragma unroll
  for (int j = 0; j < kSumPer; ++j)
    if (base + (int64_t)j * kBlock >= n) v[j] = 0.0;
  const double a = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  const double t = block_sum(a);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// One workgroup of 1024 threads; each thread keeps eight independent running
// sums (eight loads in flight) in a fixed order, so the result does not depend
// on timing.
__global__ __launch_bounds__(1024) void k_reduce_final(const double* __restrict__ partials, int64_t count,
                                                       double scale, double* __restrict__ out) {
  constexpr int kT = 1024, kU = 8;
  double acc[kU] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t i = threadIdx.x;
  for (; i + (kU - 1) * kT < count; i += kU * kT) {
#pragma unroll
    for (int u = 0; u < kU; ++u) acc[u] += partials[i + u * kT];
  }
  for (; i < count; i += kT) acc[0] += partials[i];
  const double a = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  const double t = block_sum(a);
  if (threadIdx.x == 0) out[0] = scale * t;
}

__global__ __launch_bounds__(kBlock) void k_sub_mean(int64_t n, double* __restrict__ x,
                                                     const double* __restrict__ d_mean) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] -= d_mean[0];
}

__global__ __launch_bounds__(kBlock) void k_add_correction(int64_t n, double* __restrict__ phi,
                                                           const float* __restrict__ e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) phi[i] += (double)e[i];
}

// FP64 residual of the outer defect-correction loop, rounded to FP32 per cell.
__global__ __launch_bounds__(kBlock) void k_outer_resid(int lno, double inv_h2, const double* __restrict__ phi,
                                                        const double* __restrict__ f, float* __restrict__ r32,
                                                        double* __restrict__ partials) {
  const int64_t n_oct = (int64_t)1 << (3 * lno);
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (o < n_oct) {
    const OctGeom g{lno, (1 << lno) - 1};
    int ox, oy, oz;
    oct_coords(o, lno, g.m, ox, oy, oz);
    const int64_t nb[6] = {g.idx(ox - 1, oy, oz), g.idx(ox + 1, oy, oz), g.idx(ox, oy - 1, oz),
                           g.idx(ox, oy + 1, oz), g.idx(ox, oy, oz - 1), g.idx(ox, oy, oz + 1)};
    double own[8];
    load8(phi + o * 8, own);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double s = nbr_sum(phi, own, nb, c);
      const double r = f[o * 8 + c] - (s - 6.0 * own[c]) * inv_h2;
      r32[o * 8 + c] = (float)r;
      acc += r * r;
    }
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// ---- gravitational acceleration g = -grad(phi) --------------------------
// Central differences along each axis, g_d = (phi(-e_d) - phi(+e_d)) / (2h),
// periodic wrap; with h = 1/n, 1/(2h) = n/2 is a power of two and the
// scaling is exact.  Four threads per oct, thread q holding the x-pair of
// cells 2q (cx = 0) and 2q + 1 (cx = 1) with cy = q & 1, cz = q >> 1: every
// load and store is a 16-byte pair, and a wave's stores of one component
// cover 1 KB contiguously (g is component-major [3][n_oct][8]).  Along x the
// pair's cells are each other's neighbours; along y (z) the facing pair is
// q ^ 1 (q ^ 2), in this oct on one side and in the adjacent oct on the other.
// A workgroup covers 64 consecutive octs of one x row (grids of 128^3 and
// up).  The visiting order splits the grid into slabs of 32 rows in y and
// walks each slab layer by layer in z, the 32 rows of a layer in order; with
// the workgroups numbered XCD by XCD, the rows at y +- 1 and z +- 1 were read
// by one of the last ~32 row visits of the same XCD and still sit in its L2
// (phi is fetched about once), while each layer's outputs are written as one
// contiguous run of 32 rows.  Outputs carry the streaming hint.
__global__ __launch_bounds__(kBlock) void k_force(int lno, double inv2h, const double* __restrict__ phi,
                                                  double* __restrict__ g) {
  const int64_t n_oct = (int64_t)1 << (3 * lno);
  int64_t chunk = xcd_block();                   // 64-oct chunk in visiting order
  if (lno >= 6) {
    const int ls = lno - 6;                       // log2(chunks per x row)
    const int64_t xs = chunk & ((1 << ls) - 1);
    const int64_t yy = (chunk >> ls) & 31;
    const int64_t z = (chunk >> (ls + 5)) & ((1 << lno) - 1);
    const int64_t y = ((chunk >> (ls + 5 + lno)) << 5) + yy;
    chunk = (((z << lno) + y) << ls) + xs;       // lexicographic chunk index
  }
  const int64_t t = chunk * kBlock + threadIdx.x;
  if (t >= 4 * n_oct) return;
  const int64_t o = t >> 2;
  const int q = (int)(t & 3);
  const OctGeom geo{lno, (1 << lno) - 1};
  int ox, oy, oz;
  oct_coords(o, lno, geo.m, ox, oy, oz);
  const double2* P = reinterpret_cast<const double2*>(phi);
  double2* G = reinterpret_cast<double2*>(g);
  const double2 own = P[o * 4 + q];
  const double xl = phi[geo.idx(ox - 1, oy, oz) * 8 + 2 * q + 1];
  const double xr = phi[geo.idx(ox + 1, oy, oz) * 8 + 2 * q];
  stream_store(&G[o * 4 + q], make_double2((xl - own.y) * inv2h, (own.x - xr) * inv2h));
  const bool cy = q & 1, cz = q >> 1;
  const double2 yin = P[o * 4 + (q ^ 1)];
  const double2 yout = P[geo.idx(ox, oy + (cy ? 1 : -1), oz) * 4 + (q ^ 1)];
  const double2 ylo = cy ? yin : yout, yhi = cy ? yout : yin;
  stream_store(&G[4 * n_oct + o * 4 + q], make_double2((ylo.x - yhi.x) * inv2h, (ylo.y - yhi.y) * inv2h));
  const double2 zin = P[o * 4 + (q ^ 2)];
  const double2 zout = P[geo.idx(ox, oy, oz + (cz ? 1 : -1)) * 4 + (q ^ 2)];
  const double2 zlo = cz ? zin : zout, zhi = cz ? zout : zin;
  stream_store(&G[8 * n_oct + o * 4 + q], make_double2((zlo.x - zhi.x) * inv2h, (zlo.y - zhi.y) * inv2h));
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int64_t partial_count(int64_t n_items, int block) { return (n_items + block - 1) / block; }

bool tiled_smoother(int n) { return n >= kTX && n >= kTY && n >= kTZ; }

bool small_vcycle(int n) { return n == 8 || n == 16; }

template <typename T>
void u_vcycle_small(int n0, double h0, const T* b, T* e, const T* G4, int nu_pre, int nu_post, hipStream_t s) {
  hipLaunchKernelGGL((k_vcycle_small<T>), dim3(1), dim3(1024), 0, s, n0, (T)h0, b, e, G4, nu_pre, nu_post);
  check_launch();
}

int64_t tiled_sweep_blocks(int n) { return (int64_t)(n / kTX) * (n / kTY) * (n / kTZ); }

// Number of z runs per column of the marching sweep; 0 where it is not used
// (below 256^3 a grid has too few columns to fill the chip).  Longer runs
// re-read fewer halo layers, more runs give more workgroups: the runs are
// made as long as possible (a power-of-two count) while every compute unit
// still gets two thirds of the workgroups it can hold (occupancy calculator;
// measured on 256^3: 2 of 3 per CU in f64, 4 of 6 in f32, beat both fewer and
// more).
template <typename T>
int march_runs(int n) {
  if (n < 256) return 0;
  static int target = 0;   // workgroups wanted on the device at once
  if (target == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    MG_HIP(hipGetDevice(&dev));
    MG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_smooth_march<T, false, false>,
                                                         March<T>::threads, 0));
    target = std::max(1, cus * std::max(1, 2 * per_cu / 3));
  }
  const int cols = (n / kMX) * (n / kMY);
  int runs = 1;
  while (2 * runs * cols <= target && (n / 2) / (2 * runs) >= 8) runs *= 2;
  return runs;
}

// The marching residual replaces the 3-D tile from 512^3 up, where the tile's
// re-read z halo costs HBM traffic (512^3 FP64, residual + restriction: 516
// -> 424 us; outer residual of the mixed solve: 611 -> 495 us).  At 256^3 the
// working set sits in the last-level cache and the tile is as fast (54.5 us
// against 58.2 us).
template <typename T>
int resid_march_runs(int n) {
  return n >= 512 ? march_runs<T>(n) : 0;
}

template <typename T>
int64_t u_sweep_tiled(int n, double h, const T* src, const T* b, T* dst, double* partials, hipStream_t s,
                      const T* ec_prolong, double* add64) {
  const int lno = ilog2(n / 2);
  const T h2 = (T)(h * h);
  const int runs = march_runs<T>(n);
  if (runs > 0) {
    const int64_t blocks = (int64_t)(n / kMX) * (n / kMY) * runs;
    const dim3 grid((unsigned)blocks), block(March<T>::threads);
    if (ec_prolong)
      hipLaunchKernelGGL((k_smooth_march<T, false, true>), grid, block, 0, s, lno, runs, h2, src, b, dst, partials,
                         add64, ec_prolong);
    else if (src == nullptr)
      hipLaunchKernelGGL((k_smooth_march<T, true, false>), grid, block, 0, s, lno, runs, h2, src, b, dst, partials,
                         add64, (const T*)nullptr);
    else
      hipLaunchKernelGGL((k_smooth_march<T, false, false>), grid, block, 0, s, lno, runs, h2, src, b, dst, partials,
                         add64, (const T*)nullptr);
    check_launch();
    return blocks;
  }
  const dim3 grid((unsigned)tiled_sweep_blocks(n)), block(kTileThreads);
  if (ec_prolong)
    hipLaunchKernelGGL((k_smooth_tile<T, true, false>), grid, block, 0, s, lno, h2, src, b, dst, partials, ec_prolong,
                       add64);
  else if (src == nullptr)
    hipLaunchKernelGGL((k_smooth_tile<T, false, true>), grid, block, 0, s, lno, h2, src, b, dst, partials,
                       (const T*)nullptr, add64);
  else
    hipLaunchKernelGGL((k_smooth_tile<T, false, false>), grid, block, 0, s, lno, h2, src, b, dst, partials,
                       (const T*)nullptr, add64);
  check_launch();
  return tiled_sweep_blocks(n);
}
static_assert(kTileThreads % 64 == 0 && kTileThreads <= 1024, "one workgroup (whole waves) per tile");

template <typename T>
void u_sweeps_tiled(int n, double h, T** cur, T** other, const T* b, int sweeps, bool zero_first, const T* ec,
                    hipStream_t s, double* add_last) {
  bool first = true;
  for (; sweeps > 0; --sweeps) {
    const bool last = sweeps == 1;
    u_sweep_tiled<T>(n, h, zero_first && first ? nullptr : *cur, b, *other, nullptr, s, first ? ec : nullptr,
                     last ? add_last : nullptr);
    if (!(last && add_last)) std::swap(*cur, *other);
    first = false;
  }
  if (first && zero_first) fill_zero<T>(*cur, (int64_t)n * n * n, s);   // no sweep: the zero guess itself
  if (first && ec) u_prolong<T>(n, ec, *cur, s);                        // no sweep: the prolongation alone
}

template <typename T>
void u_smooth(int n, double h, T* phi, const T* b, int sweeps, hipStream_t s, T* tmp) {
  const int lno = ilog2(n / 2);
  const int64_t n_oct = (int64_t)1 << (3 * lno);
  const T h2 = (T)(h * h);
  if (tmp != nullptr && tiled_smoother(n)) {
    T* cur = phi;
    T* other = tmp;
    u_sweeps_tiled<T>(n, h, &cur, &other, b, sweeps, false, nullptr, s);
    if (cur != phi) MG_HIP(hipMemcpyAsync(phi, cur, (size_t)n_oct * 8 * sizeof(T), hipMemcpyDeviceToDevice, s));
    return;
  }
  for (int it = 0; it < sweeps; ++it) {
    hipLaunchKernelGGL((k_smooth_colour<T, 0>), dim3(grid_for(n_oct)), dim3(kBlock), 0, s, lno, h2, phi, b);
    hipLaunchKernelGGL((k_smooth_colour<T, 1>), dim3(grid_for(n_oct)), dim3(kBlock), 0, s, lno, h2, phi, b);
  }
  check_launch();
}

template <typename T>
void u_smooth_zero_guess(int n, double h, T* phi, const T* b, int sweeps, hipStream_t s, T* tmp) {
  fill_zero(phi, (int64_t)n * n * n, s);
  u_smooth(n, h, phi, b, sweeps, s, tmp);
}

template <typename T>
int64_t u_resid_restrict(int n, double h, const T* phi, const T* b, T* bc, double* partials, hipStream_t s) {
  const int lno = ilog2(n / 2);
  const int64_t n_oct = (int64_t)1 << (3 * lno);
  const T inv_h2 = (T)(1.0 / (h * h));
  const int runs = resid_march_runs<T>(n);
  if (runs > 0) {
    const int64_t blocks = (int64_t)(n / kMX) * (n / kMY) * runs;
    const dim3 grid((unsigned)blocks), block(March<T>::threads);
    if (bc)
      hipLaunchKernelGGL((k_resid_march<T, 0>), grid, block, 0, s, lno, runs, inv_h2, phi, b, bc, (float*)nullptr,
                         partials);
    else
      hipLaunchKernelGGL((k_resid_march<T, 1>), grid, block, 0, s, lno, runs, inv_h2, phi, b, bc, (float*)nullptr,
                         partials);
    check_launch();
    return blocks;
  }
  if (tiled_smoother(n)) {
    const dim3 grid((unsigned)tiled_sweep_blocks(n)), block(kTileThreads);
    if (bc)
      hipLaunchKernelGGL((k_resid_tile<T, 0>), grid, block, 0, s, lno, inv_h2, phi, b, bc, (float*)nullptr, partials,
                         0.0, (const double*)nullptr, (double*)nullptr);
    else
      hipLaunchKernelGGL((k_resid_tile<T, 1>), grid, block, 0, s, lno, inv_h2, phi, b, bc, (float*)nullptr, partials,
                         0.0, (const double*)nullptr, (double*)nullptr);
    check_launch();
    return tiled_sweep_blocks(n);
  }
  if (bc)
    hipLaunchKernelGGL((k_resid<T, true>), dim3(grid_for(n_oct)), dim3(kBlock), 0, s, lno, inv_h2, phi, b, bc, partials);
  else
    hipLaunchKernelGGL((k_resid<T, false>), dim3(grid_for(n_oct)), dim3(kBlock), 0, s, lno, inv_h2, phi, b, bc, partials);
  check_launch();
  return partial_count(n_oct, kBlock);
}

template <typename T>
void u_prolong(int n, const T* ec, T* e, hipStream_t s) {
  const int lno = ilog2(n / 2);
  const int64_t n_oct = (int64_t)1 << (3 * lno);
  hipLaunchKernelGGL((k_prolong<T>), dim3(grid_for(n_oct)), dim3(kBlock), 0, s, lno, ec, e);
  check_launch();
}

template <typename T>
void u_coarse_solve(int n, const T* G, const T* b, T* e, hipStream_t s) {
  const int N = n * n * n;
  hipLaunchKernelGGL((k_coarse<T>), dim3(1), dim3(kBlock), 0, s, N, G, b, e);
  check_launch();
}

template <typename T>
void fill_zero(T* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_fill_zero<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, p, n);
  check_launch();
}

int64_t u_rhs(int64_t n_cells, const double* rho, const double* d_mean, double c, double* f, double* partials,
              hipStream_t s) {
  MG_REQUIRE(n_cells >= 1, "internal: right-hand side of an empty level");
  static_assert(kRhsPer == 8, "the fixed summation tree");
  const int64_t blocks = (n_cells + kBlock * kRhsPer - 1) / (kBlock * kRhsPer);
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)blocks), dim3(kBlock), 0, s, n_cells, rho, d_mean, c, f, partials);
  check_launch();
  return blocks;
}

int64_t partial_sum(int64_t n, const double* x, double* partials, hipStream_t s) {
  MG_REQUIRE(n >= 1, "internal: partial_sum of an empty array");
  static_assert(kSumPer == 8, "the fixed summation tree");
  const int64_t blocks = (n + kBlock * kSumPer - 1) / (kBlock * kSumPer);
  hipLaunchKernelGGL(k_partial_sum, dim3((unsigned)blocks), dim3(kBlock), 0, s, n, x, partials);
  check_launch();
  return blocks;
}

void reduce_final(const double* partials, int64_t count, double scale, double* out, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, s, partials, count, scale, out + slot);
  check_launch();
}

void sub_mean(int64_t n, double* x, const double* d_mean, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_mean, dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, d_mean);
  check_launch();
}

void add_correction(int64_t n, double* phi, const float* e, hipStream_t s) {
  hipLaunchKernelGGL(k_add_correction, dim3(grid_for(n)), dim3(kBlock), 0, s, n, phi, e);
  check_launch();
}

int64_t u_resid_from_rho(int n, double h, const double* phi, const double* rho, double c, const double* d_mean,
                         double* partials, double* partials_f, hipStream_t s) {
  MG_REQUIRE(tiled_smoother(n), "internal: u_resid_from_rho needs n >= 16");
  const int lno = ilog2(n / 2);
  hipLaunchKernelGGL((k_resid_tile<double, 3>), dim3((unsigned)tiled_sweep_blocks(n)), dim3(kTileThreads), 0, s, lno,
                     1.0 / (h * h), phi, rho, (double*)nullptr, (float*)nullptr, partials, c, d_mean, partials_f);
  check_launch();
  return tiled_sweep_blocks(n);
}

// From 512^3 up (FP32 arithmetic identical to the separate kernels): 512^3
// 495 + 267 -> 664 us per outer step; at 256^3, where the working set sits in
// the last-level cache, the separate tile residual and sweep are faster.
bool fused_outer_resid(int n) { return n >= 512; }

int64_t u_outer_resid_sweep(int n, double h, const double* phi, const double* f, float* r32, float* e32,
                            double* partials, hipStream_t s) {
  const int lno = ilog2(n / 2);
  const int runs = march_runs<double>(n);
  const int64_t blocks = (int64_t)(n / kMX) * (n / kMY) * runs;
  hipLaunchKernelGGL(k_outer_resid_sweep, dim3((unsigned)blocks), dim3(256), 0, s, lno, runs, 1.0 / (h * h),
                     (float)(h * h), phi, f, r32, e32, partials);
  check_launch();
  return blocks;
}

int64_t u_outer_resid(int n, double h, const double* phi, const double* f, float* r32, double* partials,
                      hipStream_t s) {
  const int lno = ilog2(n / 2);
  const int64_t n_oct = (int64_t)1 << (3 * lno);
  const int runs = resid_march_runs<double>(n);
  if (runs > 0) {
    const int64_t blocks = (int64_t)(n / kMX) * (n / kMY) * runs;
    hipLaunchKernelGGL((k_resid_march<double, 2>), dim3((unsigned)blocks), dim3(March<double>::threads), 0, s, lno,
                       runs, 1.0 / (h * h), phi, f, (double*)nullptr, r32, partials);
    check_launch();
    return blocks;
  }
  if (tiled_smoother(n)) {
    hipLaunchKernelGGL((k_resid_tile<double, 2>), dim3((unsigned)tiled_sweep_blocks(n)), dim3(kTileThreads), 0, s, lno,
                       1.0 / (h * h), phi, f, (double*)nullptr, r32, partials, 0.0, (const double*)nullptr,
                       (double*)nullptr);
    check_launch();
    return tiled_sweep_blocks(n);
  }
  hipLaunchKernelGGL(k_outer_resid, dim3(grid_for(n_oct)), dim3(kBlock), 0, s, lno, 1.0 / (h * h), phi, f, r32,
                     partials);
  check_launch();
  return partial_count(n_oct, kBlock);
}

void u_layout(int n, bool to_oct, const double* in, double* out, hipStream_t s) {
  const int lg = ilog2(n);
  if (n >= kLT) {
    const unsigned blocks = (unsigned)((n / kLT) * (n / kLT) * (n / 2));
    if (to_oct) hipLaunchKernelGGL((k_layout_tiled<true>), dim3(blocks), dim3(256), 0, s, lg, in, out);
    else hipLaunchKernelGGL((k_layout_tiled<false>), dim3(blocks), dim3(256), 0, s, lg, in, out);
  } else {
    const int64_t cells = (int64_t)n * n * n;
    if (to_oct) hipLaunchKernelGGL((k_layout_small<true>), dim3(grid_for(cells)), dim3(kBlock), 0, s, lg, in, out);
    else hipLaunchKernelGGL((k_layout_small<false>), dim3(grid_for(cells)), dim3(kBlock), 0, s, lg, in, out);
  }
  check_launch();
}

void u_force(int n, double h, const double* phi, double* g, hipStream_t s) {
  const int lno = ilog2(n / 2);
  const int64_t n_oct = (int64_t)1 << (3 * lno);
  hipLaunchKernelGGL(k_force, dim3(grid_for(4 * n_oct)), dim3(kBlock), 0, s, lno, 0.5 / h, phi, g);
  check_launch();
}

std::vector<double> coarse_pinv(int n, double h) {
  // A = F^* diag(lambda) F on the periodic grid; A^+ sums the non-zero modes:
  // A^+[p][q] = g(x_p - x_q), g(d) = (1/N) sum_{k != 0} cos(2 pi k.d / n) / lambda_k,
  // so the n^3 values of g (one per periodic offset) fill the matrix.
  const int N = n * n * n, no = n / 2;
  std::vector<int> cx(N), cy(N), cz(N);
  for (int q = 0; q < N; ++q) {
    const int o = q >> 3, c = q & 7;
    cx[q] = 2 * (o % no) + (c & 1);
    cy[q] = 2 * ((o / no) % no) + ((c >> 1) & 1);
    cz[q] = 2 * (o / (no * no)) + ((c >> 2) & 1);
  }
  const double tw = 2.0 * M_PI / n;
  std::vector<double> lam1(n);
  for (int k = 0; k < n; ++k) lam1[k] = (2.0 * std::cos(tw * k) - 2.0) / (h * h);
  std::vector<double> g((size_t)N, 0.0);
  for (int dz = 0; dz < n; ++dz)
    for (int dy = 0; dy < n; ++dy)
      for (int dx = 0; dx < n; ++dx) {
        double acc = 0.0;
        for (int kz = 0; kz < n; ++kz)
          for (int ky = 0; ky < n; ++ky)
            for (int kx = 0; kx < n; ++kx) {
              if (kx == 0 && ky == 0 && kz == 0) continue;
              const double lam = lam1[kx] + lam1[ky] + lam1[kz];
              acc += std::cos(tw * (kx * dx + ky * dy + kz * dz)) / lam;
            }
        g[((size_t)dz * n + dy) * n + dx] = acc / N;
      }
  std::vector<double> G((size_t)N * N, 0.0);
  for (int p = 0; p < N; ++p)
    for (int q = 0; q < N; ++q) {
      const int dx = ((cx[p] - cx[q]) % n + n) % n, dy = ((cy[p] - cy[q]) % n + n) % n,
                dz = ((cz[p] - cz[q]) % n + n) % n;
      G[(size_t)p * N + q] = g[((size_t)dz * n + dy) * n + dx];
    }
  return G;
}

#define MG_INST(T)                                                                                 \
  template void u_smooth<T>(int, double, T*, const T*, int, hipStream_t, T*);                      \
  template int64_t u_sweep_tiled<T>(int, double, const T*, const T*, T*, double*, hipStream_t, const T*, double*); \
  template void u_sweeps_tiled<T>(int, double, T**, T**, const T*, int, bool, const T*, hipStream_t, double*); \
  template void u_vcycle_small<T>(int, double, const T*, T*, const T*, int, int, hipStream_t);      \
  template void u_smooth_zero_guess<T>(int, double, T*, const T*, int, hipStream_t, T*);           \
  template int64_t u_resid_restrict<T>(int, double, const T*, const T*, T*, double*, hipStream_t); \
  template void u_prolong<T>(int, const T*, T*, hipStream_t);                                      \
  template void u_coarse_solve<T>(int, const T*, const T*, T*, hipStream_t);                       \
  template void fill_zero<T>(T*, int64_t, hipStream_t);
MG_INST(double)
MG_INST(float)
#undef MG_INST

}  // namespace mg

// Kernels for levels made of an arbitrary set of octs (refined levels and the
// father-cell multigrid hierarchy below them).
//
// * Morton key of oct coordinates (equation morton_encode): bit b of x, y, z
//   goes to key bit 3b, 3b+1, 3b+2 (21 bits per axis, bit 63 unused).  Computed
//   here with the usual shift-and-mask bit spreading.
// * Open-addressing hash table (appendix "Per-level hash table and replacement
//   functions", equation hash_func): t = ((k * phi1) ^ (k >> 16)) * phi2,
//   h = t ^ (t >> 13) in unsigned 64-bit arithmetic, slot = h & (capacity - 1),
//   linear probing; insertion claims a slot with a 64-bit compare-and-swap.
// * Neighbour cache (equation nbor_precompute): six neighbour oct indices per
//   oct, looked up once per build (neighbour key = key of the coordinates
//   stepped by one with periodic wrap, algorithm "Morton neighbour key").
// * Parent keys are key >> 3 and the low three key bits are the child index
//   cx + 2cy + 4cz, which is also the oct-major cell index.
#include <hipcub/hipcub.hpp>

#include "mg_internal.h"

namespace mg {

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kEmpty = ~0ull;

struct Slot {
  unsigned long long key;
  int32_t val;
  int32_t pad;
};

__device__ __forceinline__ int32_t hash_lookup(const Slot* __restrict__ t, uint64_t mask, uint64_t k) {
  uint64_t s = hash64(k) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long kk = t[s].key;
    if (kk == k) return t[s].val;
    if (kk == kEmpty) return -1;
    s = (s + 1) & mask;
  }
  return -1;
}

__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t* __restrict__ a, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ int32_t find_sorted(const uint64_t* __restrict__ a, int64_t n, uint64_t k) {
  const int64_t p = lower_bound_u64(a, n, k);
  return (p < n && a[p] == k) ? (int32_t)p : -1;
}

// cell c's slot among the four cells of the face it touches along axis d
__device__ __forceinline__ int face_slot(int c, int d) {
  return d == 0 ? (c >> 1) : (d == 1 ? ((c & 1) | ((c >> 2) << 1)) : (c & 3));
}
__device__ __forceinline__ int face_cell(int k, int d, int side) {
  return d == 0 ? (side | (k << 1)) : (d == 1 ? ((k & 1) | (side << 1) | ((k >> 1) << 2)) : (k | (side << 2)));
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// build kernels
// ---------------------------------------------------------------------------
__global__ void k_morton(int64_t n, const int32_t* __restrict__ ijk, uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = morton((uint32_t)ijk[3 * i], (uint32_t)ijk[3 * i + 1], (uint32_t)ijk[3 * i + 2]);
}

__global__ void k_validate(int64_t n, const int32_t* __restrict__ ijk, int n_dim, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int d = 0; d < 3; ++d) {
    const int v = ijk[3 * i + d];
    if (v < 0 || v >= n_dim) atomicOr(flag, 1);
  }
}

__global__ void k_hash_clear(int64_t cap, Slot* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cap) {
    t[i].key = kEmpty;
    t[i].val = -1;
    t[i].pad = 0;
  }
}

__global__ void k_hash_insert(int64_t n, const uint64_t* __restrict__ keys, Slot* __restrict__ t, uint64_t mask,
                              int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long k = keys[i];
  uint64_t s = hash64(k) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev = atomicCAS(&t[s].key, kEmpty, k);
    if (prev == kEmpty) {
      t[s].val = (int32_t)i;
      return;
    }
    if (prev == k) {
      atomicOr(flag, 2);  // duplicate oct
      return;
    }
    s = (s + 1) & mask;
  }
  atomicOr(flag, 4);  // table full
}

__global__ void k_hash_lookup(int64_t n, const uint64_t* __restrict__ q, const Slot* __restrict__ t, uint64_t mask,
                              int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = hash_lookup(t, mask, q[i]);
}

// neighbour cache of the finest level via the hash table: eight lanes per oct
// (face j = lane & 7 below 6, one lookup each), the oct's missing faces
// counted across its lanes
__global__ void k_nbr_hash(int64_t n, const uint64_t* __restrict__ keys, int n_dim, const Slot* __restrict__ t,
                           uint64_t mask, int32_t* __restrict__ nbr, int32_t* __restrict__ missing) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = u >> 3;
  const int j = (int)(u & 7);
  int miss = 0;
  if (i < n && j < 6) {
    int x, y, z;
    unmorton(keys[i], x, y, z);
    const int m = n_dim - 1;  // n_dim is a power of two
    const int d = j >> 1, st = (j & 1) ? 1 : -1;
    const int xx = (x + (d == 0 ? st : 0)) & m, yy = (y + (d == 1 ? st : 0)) & m, zz = (z + (d == 2 ? st : 0)) & m;
    const int32_t v = hash_lookup(t, mask, morton(xx, yy, zz));
    nbr[i * 6 + j] = v;
    miss = v < 0;
  }
  // the 8 lanes of an oct are an aligned group of the wave
  miss += __shfl_xor(miss, 1, 64);
  miss += __shfl_xor(miss, 2, 64);
  miss += __shfl_xor(miss, 4, 64);
  if (i < n && j == 0) missing[i] = miss;
}

// number the ghost faces, mark them in nbr as -2 - g and record each ghost
// cell's 8 coarse interpolation cells on the parent level
// A level's keys hold oct coordinates in its key frame (see mg_level_s);
// frame_shift[a] = (this level's frame origin in octs) - 2 (the parent's frame
// origin in octs) converts this level's relative oct coordinate into the
// parent's relative cell coordinate; pcells is the parent's cell extent of
// its key space (a power of two; parent coordinates wrap modulo it).
__global__ void k_ghost_stencil(int64_t n, const uint64_t* __restrict__ keys, int n_dim,
                                const int32_t* __restrict__ first, int32_t* __restrict__ nbr,
                                int parent_uniform, const Slot* __restrict__ pt, uint64_t pmask,
                                int pcells, int sx, int sy, int sz,
                                int32_t* __restrict__ gidx, int* __restrict__ flag) {
  // eight lanes per oct (an aligned group of the wave), lane j < 6 for face j
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = u >> 3;
  const int j = (int)(u & 7);
  const bool valid = i < n && j < 6;
  const bool miss = valid && nbr[i * 6 + j] < 0;
  // every lane has read its face before any lane writes: ghost numbers follow
  // the oct's missing faces in face order
  const unsigned long long bal = __ballot(miss);
  if (!miss) return;
  const int lane = (int)(threadIdx.x & 63);
  const unsigned long long group_below = bal & ((1ull << lane) - 1ull) & (0xFFull << (lane & ~7));
  const int g = first[i] + __popcll(group_below);
  nbr[i * 6 + j] = -2 - g;
  int x, y, z;
  unmorton(keys[i], x, y, z);
  const int ncell = 2 * n_dim;          // this level's cells per dimension (key frame)
  const int pm = pcells - 1;            // parent cells per dimension - 1
  const int pom = (pcells >> 1) - 1;    // parent octs per dimension - 1
  const int pno_log = __ffs(pcells) - 1 - 1;   // log2(parent octs per dimension) (uniform parent)
  const int shift[3] = {sx, sy, sz};
  const int d = j >> 1, side = j & 1, st = side ? 1 : -1;
  // each of the face's 4 ghost cells interpolates from 8 parent cells P + {0, s} per axis
  int P[4][3], sg[4][3];
  int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = face_cell(k, d, side);
    int gc[3] = {2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1)};
    gc[d] = (gc[d] + st + ncell) & (ncell - 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      P[k][a] = (gc[a] >> 1) + shift[a];
      sg[k][a] = (gc[a] & 1) ? 1 : -1;
      lo[a] = min(lo[a], P[k][a] - (sg[k][a] < 0 ? 1 : 0));
    }
  }
  // the parent cells span at most 3 per axis, so at most 2 parent octs per
  // axis, from (lo >> 1): the 8 candidate octs, looked up once each
  int32_t po8[8];
  if (!parent_uniform) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t ox = (uint32_t)(((lo[0] >> 1) + (e & 1)) & pom), oy = (uint32_t)(((lo[1] >> 1) + ((e >> 1) & 1)) & pom),
                     oz = (uint32_t)(((lo[2] >> 1) + (e >> 2)) & pom);
      po8[e] = hash_lookup(pt, pmask, morton(ox, oy, oz));
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int a = (q >> 2) & 1, b = (q >> 1) & 1, cc = q & 1;   // q = 4a + 2b + c, a along x
      const int X = P[k][0] + a * sg[k][0], Y = P[k][1] + b * sg[k][1], Z = P[k][2] + cc * sg[k][2];
      const int child = (X & 1) + 2 * (Y & 1) + 4 * (Z & 1);
      int32_t po;
      if (parent_uniform) {
        po = (int32_t)(((((int64_t)((Z & pm) >> 1) << pno_log) + ((Y & pm) >> 1)) << pno_log) + ((X & pm) >> 1));
      } else {
        po = po8[((X >> 1) - (lo[0] >> 1)) + 2 * ((Y >> 1) - (lo[1] >> 1)) + 4 * ((Z >> 1) - (lo[2] >> 1))];
      }
      if (po < 0) {
        atomicOr(flag, 8);
        po = 0;
      }
      gidx[((int64_t)g * 4 + k) * 8 + q] = po * 8 + child;
    }
  }
}

// Level-set mask of the coarse multigrid levels of a refined level.  Every
// cell of the finest level has mask +1; a coarse father cell takes the mean
// of its 8 children's masks, every other coarse cell -1.  A cell is active
// (an unknown of the coarse error equation) when its mask is positive.  For
// an active cell c and an inactive or absent neighbour j, the zero of the
// error lies where the mask interpolates to zero between the two centres, at
// fraction theta = m_c / (m_c - m_j) (clamped to [0.1, 1]); extrapolating e
// linearly through that zero gives e_j = e_c (1 - 1/theta), so the cell's
// diagonal becomes 6 + sum_j (1/theta_j - 1).  With m_c = 1, m_j = -1 the zero
// is on the shared face (e_j = -e_c).
__global__ void k_fill_f32(int64_t n, float v, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

__global__ void k_coarse_lsm(int64_t n_fine, const int32_t* __restrict__ father, const float* __restrict__ fine_lsm,
                             float* __restrict__ coarse_lsm) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_fine) return;
  float m = 1.0f;
  if (fine_lsm) {
    float acc = 0.0f;
    for (int c = 0; c < 8; ++c) acc += fine_lsm[o * 8 + c];
    m = acc * 0.125f;
  }
  coarse_lsm[father[o]] = m;
}

template <typename T>
__global__ void k_lsm_operator(int64_t n, const int32_t* __restrict__ nbr, const float* __restrict__ lsm,
                               uint8_t* __restrict__ mask, T* __restrict__ diag) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  unsigned bits = 0;
  for (int c = 0; c < 8; ++c) {
    const float mc = lsm[o * 8 + c];
    double d = 6.0;
    if (mc > 0.0f) {
      bits |= 1u << c;
      for (int d3 = 0; d3 < 3; ++d3) {
        const int cn = c ^ (1 << d3);
        // neighbour inside the oct, then across the face on the side of bit d3 of c
        const float m_in = lsm[o * 8 + cn];
        const int v = nbr[o * 6 + 2 * d3 + ((c >> d3) & 1)];
        const float m_out = v >= 0 ? lsm[(int64_t)v * 8 + cn] : -1.0f;
        const float mj[2] = {m_in, m_out};
        for (int t = 0; t < 2; ++t) {
          if (mj[t] > 0.0f) continue;
          double th = (double)mc / ((double)mc - (double)mj[t]);
          th = th < 0.1 ? 0.1 : (th > 1.0 ? 1.0 : th);
          d += 1.0 / th - 1.0;
        }
      }
    }
    diag[o * 8 + c] = (T)d;
  }
  mask[o] = (uint8_t)bits;
}

__global__ void k_nbr_export(int64_t n6, const int32_t* __restrict__ nbr, int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n6) out[i] = nbr[i] >= 0 ? nbr[i] : -1;
}

// ancestor keys: key >> drop (3 per level up)
__global__ void k_parent_keys(int64_t n, const uint64_t* __restrict__ keys, int drop, uint64_t* __restrict__ pk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pk[i] = keys[i] >> drop;
}

// flat index of each oct's father cell on the coarse level
__global__ void k_fathers(int64_t n, const uint64_t* __restrict__ keys, const uint64_t* __restrict__ ckeys,
                          int64_t nc, int32_t* __restrict__ father, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = keys[i];
  const int32_t co = find_sorted(ckeys, nc, k >> 3);
  if (co < 0) {
    atomicOr(flag, 16);
    father[i] = 0;
    return;
  }
  father[i] = co * 8 + (int)(k & 7);
}

// the 27-neighbourhood of each oct of a sorted level, one search per thread
// (27 threads per oct); the face neighbours are its entries with one nonzero offset
__global__ void k_nbr_sorted(int64_t n, const uint64_t* __restrict__ keys, int n_dim, int32_t* __restrict__ nbr,
                             int32_t* __restrict__ nbr27) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n * 27) return;
  const int64_t i = u / 27;
  const int q = (int)(u - i * 27);
  int x, y, z;
  unmorton(keys[i], x, y, z);
  const int m = n_dim - 1;
  const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
  const int32_t v = find_sorted(keys, n, morton((x + dx) & m, (y + dy) & m, (z + dz) & m));
  nbr27[u] = v;
  if ((dx != 0) + (dy != 0) + (dz != 0) == 1) {
    const int dd = dx != 0 ? 0 : (dy != 0 ? 1 : 2);
    nbr[i * 6 + 2 * dd + (dx + dy + dz > 0 ? 1 : 0)] = v;
  }
}

// ---------------------------------------------------------------------------
// solve kernels on oct levels
// ---------------------------------------------------------------------------
// Sum of the six neighbours of cell c; absent neighbours count 0, ghosts
// (finest level, GHOST) come from the ghost array.
template <typename T, bool GHOST>
__device__ __forceinline__ T oct_nbr_sum(const T* __restrict__ e, const T (&own)[8], const int32_t (&nb)[6],
                                         const double* __restrict__ ghost, int c) {
  T s = own[c ^ 1] + own[c ^ 2] + own[c ^ 4];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int v = nb[2 * d + ((c >> d) & 1)];
    if (v >= 0) s += e[(int64_t)v * 8 + (c ^ (1 << d))];
    else if (GHOST && v <= -2) s += (T)ghost[(int64_t)(-2 - v) * 4 + face_slot(c, d)];
  }
  return s;
}

template <typename T, int COLOUR, bool GHOST>
__global__ __launch_bounds__(kBlock) void k_oct_smooth(int64_t n, T h2, T* __restrict__ e, const T* __restrict__ b,
                                                       const int32_t* __restrict__ nbr,
                                                       const uint8_t* __restrict__ mask,
                                                       const T* __restrict__ diag,
                                                       const double* __restrict__ ghost) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const unsigned mk = mask ? mask[o] : 0xFFu;
  int32_t nb[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) nb[j] = nbr[o * 6 + j];
  T own[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) own[c] = e[o * 8 + c];
  const T sixth = T(1) / T(6);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (((c ^ (c >> 1) ^ (c >> 2)) & 1) != COLOUR || !((mk >> c) & 1u)) continue;
    const T s = oct_nbr_sum<T, GHOST>(e, own, nb, ghost, c);
    const T inv_diag = diag ? T(1) / diag[o * 8 + c] : sixth;
    e[o * 8 + c] = (s - h2 * b[o * 8 + c]) * inv_diag;
  }
}

// residual on active cells (+ restriction to the father cell, + per-cell f32 copy)
template <typename T, bool GHOST, bool RESTRICT>
__global__ __launch_bounds__(kBlock) void k_oct_resid(int64_t n, T inv_h2, const T* __restrict__ e,
                                                      const T* __restrict__ b, const int32_t* __restrict__ nbr,
                                                      const uint8_t* __restrict__ mask,
                                                      const T* __restrict__ diag,
                                                      const double* __restrict__ ghost,
                                                      const int32_t* __restrict__ father, T* __restrict__ bc,
                                                      float* __restrict__ r32, double* __restrict__ partials) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (o < n) {
    const unsigned mk = mask ? mask[o] : 0xFFu;
    int32_t nb[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) nb[j] = nbr[o * 6 + j];
    T own[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) own[c] = e[o * 8 + c];
    T rsum = T(0);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      T r = T(0);
      if ((mk >> c) & 1u) {
        const T s = oct_nbr_sum<T, GHOST>(e, own, nb, ghost, c);
        const T dg = diag ? diag[o * 8 + c] : T(6);
        r = b[o * 8 + c] - (s - dg * own[c]) * inv_h2;
      }
      if (r32) r32[o * 8 + c] = (float)r;
      rsum += r;
      acc += (double)r * (double)r;
    }
    if (RESTRICT && father[o] >= 0) bc[father[o]] = rsum * T(0.125);
  }
  if (partials) {
    const double t = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
  }
}

// g = -grad(phi) on the finest level by central differences: a face
// neighbour is the adjacent oct's cell, or (ghost face) the interpolated
// parent value the solve uses.  Component-major output [3][n][8]; four
// threads per oct, each on an x-pair of cells (the periodic kernel's layout).
__device__ __forceinline__ double across_face(const double* __restrict__ phi, const double* __restrict__ ghost,
                                              int v, int cell_there, int c, int d) {
  if (v >= 0) return phi[(int64_t)v * 8 + cell_there];
  if (v <= -2) return ghost[(int64_t)(-2 - v) * 4 + face_slot(c, d)];
  return 0.0;   // absent: does not occur on a finest level, where every open face has a ghost
}

__global__ __launch_bounds__(kBlock) void k_oct_force(int64_t n, double inv2h, const double* __restrict__ phi,
                                                      const int32_t* __restrict__ nbr,
                                                      const double* __restrict__ ghost, double* __restrict__ g) {
  const int64_t t = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
  if (t >= 4 * n) return;
  const int64_t o = t >> 2;
  const int q = (int)(t & 3);
  const int c0 = 2 * q, c1 = 2 * q + 1;
  const double2* P = reinterpret_cast<const double2*>(phi);
  double2* G = reinterpret_cast<double2*>(g);
  const double2 own = P[o * 4 + q];
  const double xl = across_face(phi, ghost, nbr[o * 6 + 0], c1, c0, 0);
  const double xr = across_face(phi, ghost, nbr[o * 6 + 1], c0, c1, 0);
  stream_store(&G[o * 4 + q], make_double2((xl - own.y) * inv2h, (own.x - xr) * inv2h));
  const bool cy = q & 1, cz = q >> 1;
  const double2 yin = P[o * 4 + (q ^ 1)];
  const int vy = nbr[o * 6 + (cy ? 3 : 2)];
  const double2 yout = vy >= 0 ? P[(int64_t)vy * 4 + (q ^ 1)]
                               : make_double2(across_face(phi, ghost, vy, 0, c0, 1), across_face(phi, ghost, vy, 0, c1, 1));
  const double2 ylo = cy ? yin : yout, yhi = cy ? yout : yin;
  stream_store(&G[4 * n + o * 4 + q], make_double2((ylo.x - yhi.x) * inv2h, (ylo.y - yhi.y) * inv2h));
  const double2 zin = P[o * 4 + (q ^ 2)];
  const int vz = nbr[o * 6 + (cz ? 5 : 4)];
  const double2 zout = vz >= 0 ? P[(int64_t)vz * 4 + (q ^ 2)]
                               : make_double2(across_face(phi, ghost, vz, 0, c0, 2), across_face(phi, ghost, vz, 0, c1, 2));
  const double2 zlo = cz ? zin : zout, zhi = cz ? zout : zin;
  stream_store(&G[8 * n + o * 4 + q], make_double2((zlo.x - zhi.x) * inv2h, (zlo.y - zhi.y) * inv2h));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_oct_prolong(int64_t n, const int32_t* __restrict__ father,
                                                        const int32_t* __restrict__ cnbr27, const T* __restrict__ ec,
                                                        T* __restrict__ e, const uint8_t* __restrict__ mask) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int32_t F = father[o];
  const int32_t O = F >> 3;
  const int cf = F & 7;
  const int fx = cf & 1, fy = (cf >> 1) & 1, fz = cf >> 2;
  T E[3][3][3];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int tx = fx + dx, ty = fy + dy, tz = fz + dz;          // in [-1, 2]
        const int q = ((tz >> 1) + 1) * 9 + ((ty >> 1) + 1) * 3 + ((tx >> 1) + 1);
        const int32_t co = cnbr27[(int64_t)O * 27 + q];
        E[dz + 1][dy + 1][dx + 1] = co >= 0 ? ec[(int64_t)co * 8 + (tx & 1) + 2 * (ty & 1) + 4 * (tz & 1)] : T(0);
      }
  const unsigned mk = mask ? mask[o] : 0xFFu;
  const T w[2] = {T(0.75), T(0.25)};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (!((mk >> c) & 1u)) continue;
    const int sx = (c & 1) ? 1 : -1, sy = (c & 2) ? 1 : -1, sz = (c & 4) ? 1 : -1;
    T v = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) v += (w[a] * w[bb] * w[cc]) * E[1 + cc * sz][1 + bb * sy][1 + a * sx];
    e[o * 8 + c] += v;
  }
}

// ---------------------------------------------------------------------------
// Brick sweeps: one fused red + black sweep per launch on LDS-staged oct
// neighbourhoods.  The octs of a level are grouped in bricks of 4 x 4 x 4 octs
// on a lattice shifted by 0 or 1 oct along each axis (the level's brick shift,
// bit a for axis a: brick = (oct + shift) >> 2, chosen per level for the
// fewest bricks); a workgroup of 64 threads (one oct each) stages its brick and a
// one-oct halo (6 x 6 x 6 octs = 12^3 cells, through the brick map built at
// level build time), writes the Dirichlet ghost values of absent neighbours
// into the box (finest level), updates the red cells of the brick and of the
// one-cell ring around it (the ring's red values are exactly what the
// neighbouring bricks compute), then the black cells of the brick, and writes
// the brick's octs to the other buffer.  Absent octs count 0 (coarse levels)
// or supply ghosts; inactive cells keep their value.
// ---------------------------------------------------------------------------
constexpr int kBrickOcts = 64;            // 4 x 4 x 4
constexpr int kBoxOcts = 216;             // 6 x 6 x 6
constexpr int kBoxCells = 12;             // cells per box edge
constexpr int kBrickShell = 244;          // red cells of the one-cell ring around the 8^3 brick cells
constexpr int kCoarseBoxOcts = 125;       // 5 x 5 x 5 coarse octs holding a brick's 8^3 coarse window
// the shift is chosen on levels of at least this many octs and at most this
// many octs per dimension (8 bitmaps of (n_dim / 4)^3 bits: 16 MiB at 1024)
constexpr int64_t kBrickShiftMinOcts = 4096;
constexpr int kBrickShiftMaxDim = 1024;
struct BrickShell {
  uint16_t v[kBrickShell];                // box cell index (z * 12 + y) * 12 + x
};
constexpr BrickShell make_brick_shell() {
  BrickShell t{};
  int k = 0;
  for (int z = 1; z < 11; ++z)
    for (int y = 1; y < 11; ++y)
      for (int x = 1; x < 11; ++x) {
        const bool inner = x >= 2 && x < 10 && y >= 2 && y < 10 && z >= 2 && z < 10;
        if (!inner && ((x + y + z) & 1) == 0) t.v[k++] = (uint16_t)((z * 12 + y) * 12 + x);
      }
  return t;
}
__constant__ BrickShell kBrickShellCells = make_brick_shell();

// map[b][q] = index of the oct at brick b's box position q = (qz * 6 + qy) * 6 + qx
// (oct coordinates 4 bx - 1 - sx + qx, ... with periodic wrap, (sx, sy, sz) the
// level's brick shift), -1 if absent
__global__ void k_brick_map(int64_t n_bricks, const uint64_t* __restrict__ bkeys, int n_dim, int shift,
                            const Slot* __restrict__ table, uint64_t tmask, const uint64_t* __restrict__ skeys,
                            int64_t n_sorted, int32_t* __restrict__ map) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_bricks * kBoxOcts) return;
  const int64_t bidx = i / kBoxOcts;
  const int q = (int)(i % kBoxOcts);
  int bx, by, bz;
  unmorton(bkeys[bidx], bx, by, bz);
  const int m = n_dim - 1;
  const uint32_t x = (uint32_t)((4 * bx - 1 - (shift & 1) + q % 6) & m),
                 y = (uint32_t)((4 * by - 1 - ((shift >> 1) & 1) + (q / 6) % 6) & m),
                 z = (uint32_t)((4 * bz - 1 - (shift >> 2) + q / 36) & m);
  const uint64_t k = morton(x, y, z);
  map[i] = table ? hash_lookup(table, tmask, k) : find_sorted(skeys, n_sorted, k);
}

// cmap[b][u] = index of the coarse oct at position u = (w * 5 + v) * 5 + u0 of
// brick b's coarse box (coarse oct coordinates 2 bx - 1 - sx + u0, ... with
// periodic wrap on the coarse level), -1 if absent or outside the window.  The
// box's octs have their fathers at coarse cells 4 bx - 1 - sx + q (q = 0..5)
// and a prolongation into them reads the coarse cells one further out: the 8
// cells from 4 bx - 2 - sx per axis, the window, which starts in the first
// coarse oct of the box (cell 1 of it when sx = 1) and ends in its fourth
// (sx = 0: the fifth oct is outside, and marked absent) or fifth.
__global__ void k_brick_cmap(int64_t n_bricks, const uint64_t* __restrict__ bkeys, int n_dim_c, int shift,
                             const uint64_t* __restrict__ ckeys, int64_t n_coarse, int32_t* __restrict__ cmap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_bricks * kCoarseBoxOcts) return;
  const int u = (int)(i % kCoarseBoxOcts);
  const int ux = u % 5, uy = (u / 5) % 5, uz = u / 25;
  const int sx = shift & 1, sy = (shift >> 1) & 1, sz = shift >> 2;
  if ((ux == 4 && !sx) || (uy == 4 && !sy) || (uz == 4 && !sz)) {
    cmap[i] = -1;
    return;
  }
  int bx, by, bz;
  unmorton(bkeys[i / kCoarseBoxOcts], bx, by, bz);
  const int m = n_dim_c - 1;
  const uint32_t x = (uint32_t)((2 * bx - 1 - sx + ux) & m), y = (uint32_t)((2 * by - 1 - sy + uy) & m),
                 z = (uint32_t)((2 * bz - 1 - sz + uz) & m);
  cmap[i] = find_sorted(ckeys, n_coarse, morton(x, y, z));
}

// Brick shift selection: lattice j (shift j) owns words [j * words_per,
// (j + 1) * words_per); bit (bz * nb + by) * nb + bx of them marks brick
// (bx, by, bz) as holding an oct
__global__ void k_brick_shift_bits(int64_t n, const uint64_t* __restrict__ keys, int n_dim, int64_t words_per,
                                   uint32_t* __restrict__ bits) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  int x = 0, y = 0, z = 0;
  if (valid) unmorton(keys[i], x, y, z);
  const int m = n_dim - 1, nb = n_dim >> 2;
  const int lane = (int)(threadIdx.x & 63);
  for (int j = 0; j < 8; ++j) {
    const int64_t bx = ((x + (j & 1)) & m) >> 2, by = ((y + ((j >> 1) & 1)) & m) >> 2, bz = ((z + (j >> 2)) & m) >> 2;
    const int64_t bit = valid ? (bz * nb + by) * nb + bx : -1;
    // octs of a brick mostly come in runs: the first lane of a run sets the bit
    const int64_t prev = __shfl_up(bit, 1, 64);
    if (valid && (lane == 0 || prev != bit)) atomicOr(bits + j * words_per + (bit >> 5), 1u << (bit & 31));
  }
}
// counts[j] += set bits of lattice j's words (per-workgroup partial sums)
__global__ __launch_bounds__(kBlock) void k_brick_shift_count(int64_t words_per, const uint32_t* __restrict__ bits,
                                                               unsigned long long* __restrict__ counts) {
  const int j = blockIdx.y;
  unsigned long long c = 0;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words_per; w += (int64_t)gridDim.x * blockDim.x)
    c += __popc(bits[j * words_per + w]);
  __shared__ unsigned long long red[kBlock];
  red[threadIdx.x] = c;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(counts + j, red[0]);
}
// keys of the shifted oct coordinates ((x + sx) & m, ...)
__global__ void k_shift_keys(int64_t n, const uint64_t* __restrict__ keys, int n_dim, int shift,
                             uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int x, y, z;
  unmorton(keys[i], x, y, z);
  const int m = n_dim - 1;
  out[i] = morton((uint32_t)((x + (shift & 1)) & m), (uint32_t)((y + ((shift >> 1) & 1)) & m),
                  (uint32_t)((z + (shift >> 2)) & m));
}

// Ghost lists: for each brick, the box cells that hold a Dirichlet ghost
// (cells of absent octs next to a ghost face of a present oct of the box) and
// the ghost value each takes (flat index g * 4 + face slot).  A ghost value
// depends only on its cell's position, so two faces that name the same cell
// name the same value.  Built in two passes (count, then fill at the scanned
// offsets) over (brick, box oct) pairs.
__device__ __forceinline__ int brick_ghost_scan(const int32_t* __restrict__ bm, const int32_t* __restrict__ nbr,
                                                int q, int32_t* __restrict__ cell, int32_t* __restrict__ gv) {
  const int32_t o = bm[q];
  if (o < 0) return 0;
  const int qx = q % 6, qy = (q / 6) % 6, qz = q / 36;
  int cnt = 0;
  for (int j = 0; j < 6; ++j) {
    const int32_t nv = nbr[(int64_t)o * 6 + j];
    if (nv > -2) continue;
    const int g = -2 - nv, d = j >> 1, side = j & 1;
    for (int k = 0; k < 4; ++k) {
      const int c = face_cell(k, d, side);
      int x = 2 * qx + (c & 1), y = 2 * qy + ((c >> 1) & 1), z = 2 * qz + (c >> 2);
      const int step = side ? 1 : -1;
      if (d == 0) x += step;
      else if (d == 1) y += step;
      else z += step;
      if (x < 0 || x >= kBoxCells || y < 0 || y >= kBoxCells || z < 0 || z >= kBoxCells) continue;
      if (cell) {
        cell[cnt] = (z * kBoxCells + y) * kBoxCells + x;
        gv[cnt] = g * 4 + k;
      }
      ++cnt;
    }
  }
  return cnt;
}
__global__ void k_brick_ghost_count(int64_t n_bricks, const int32_t* __restrict__ map, const int32_t* __restrict__ nbr,
                                    int32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_bricks * kBoxOcts) return;
  count[i] = brick_ghost_scan(map + (i / kBoxOcts) * kBoxOcts, nbr, (int)(i % kBoxOcts), nullptr, nullptr);
}
__global__ void k_brick_ghost_fill(int64_t n_bricks, const int32_t* __restrict__ map, const int32_t* __restrict__ nbr,
                                   const int32_t* __restrict__ first, int32_t* __restrict__ cell,
                                   int32_t* __restrict__ gv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_bricks * kBoxOcts) return;
  brick_ghost_scan(map + (i / kBoxOcts) * kBoxOcts, nbr, (int)(i % kBoxOcts), cell + first[i], gv + first[i]);
}

// 16-byte pieces of one oct's 8 values
template <typename T> struct OctVec;
template <> struct OctVec<double> { using V = double2; static constexpr int n = 2; };
template <> struct OctVec<float> { using V = float4; static constexpr int n = 4; };
template <typename T>
__device__ __forceinline__ void load_oct(const T* __restrict__ p, T (&v)[8]) {
  using V = typename OctVec<T>::V;
  constexpr int VN = OctVec<T>::n;
#pragma unroll
  for (int k = 0; k < 8 / VN; ++k) {
    const V x = reinterpret_cast<const V*>(p)[k];
    const T* px = reinterpret_cast<const T*>(&x);
#pragma unroll
    for (int j = 0; j < VN; ++j) v[k * VN + j] = px[j];
  }
}
template <typename T>
__device__ __forceinline__ void store_oct(T* __restrict__ p, const T (&v)[8]) {
  using V = typename OctVec<T>::V;
  constexpr int VN = OctVec<T>::n;
#pragma unroll
  for (int k = 0; k < 8 / VN; ++k) {
    V x;
    T* px = reinterpret_cast<T*>(&x);
#pragma unroll
    for (int j = 0; j < VN; ++j) px[j] = v[k * VN + j];
    reinterpret_cast<V*>(p)[k] = x;
  }
}

// A brick is worked by 8 / R threads per oct: thread t owns the R cells
// c = c0 + k (k < R, c0 = R (t mod 8/R)) of the brick's oct t / (8/R) (R = 4:
// one cell plane cz, R = 2: one row (cy, cz)), so several waves share one box
// of LDS and each stages and updates a part of it.  Cells per thread of each
// brick kernel, as measured on a 5.1M-cell refined level (FP64 solve: one
// wave per brick 6.84 ms, R = 4 6.15 ms, plain sweeps at R = 2 6.09 ms; R = 2
// for the FP32 kernels, whose box takes half the LDS, leaves fewer bricks per
// compute unit under the wave limit and was slower, as was the residual at
// R = 2):
template <typename T> constexpr int kSweepCells = sizeof(T) == 8 ? 2 : 4;
constexpr int kProlongCells = 4, kResidCells = 4;
template <int R> struct BrickShape {
  static_assert(R == 2 || R == 4, "two or four cells per thread");
  static constexpr int G = 8 / R;                                    // threads per oct
  static constexpr int NT = kBrickOcts * G;                          // threads per brick
  static constexpr int StagePer = (kBoxOcts + NT - 1) / NT;          // box octs staged per thread
  static constexpr int GhostPer = NT >= 256 ? 1 : 256 / NT;          // ghost-list entries held in registers
  static constexpr int ShellPer = (kBrickShell + NT - 1) / NT;       // red ring cells per thread
};

// A brick's box (12^3 cells) on its way into LDS.  The loads go out in two
// batches: the map entries (and the bounds of the brick's ghost list), then
// every value (the box octs' values and the ghost cells with their values,
// gathered per solve in list order), so a workgroup waits for two memory
// round trips instead of a chain of dependent ones.  On the finest level
// (GHOST) the cells of absent octs are not zeroed: every one of them that an
// update reads is a ghost cell, written from the list.
template <typename T, bool ZERO, bool GHOST, int R>
struct BrickBox {
  using S = BrickShape<R>;
  int32_t oq[S::StagePer];
  T v[S::StagePer][8];
  int g0 = 0, g1 = 0;
  int gc[S::GhostPer];
  T gv[S::GhostPer];

  __device__ __forceinline__ void load_map(const int32_t* __restrict__ bm, const int32_t* __restrict__ gfirst,
                                           int64_t brick) {
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < S::StagePer; ++r) {
      const int q = t + r * S::NT;
      oq[r] = q < kBoxOcts ? bm[q] : -1;
    }
    if (GHOST) {
      g0 = gfirst[brick * kBoxOcts];
      g1 = gfirst[(brick + 1) * kBoxOcts];
    }
  }
  __device__ __forceinline__ void load_values(const T* __restrict__ src, const int32_t* __restrict__ gcell,
                                              const double* __restrict__ gval) {
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < S::StagePer; ++r) {
      if (!ZERO && oq[r] >= 0) {
        load_oct(src + (int64_t)oq[r] * 8, v[r]);
      } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) v[r][c] = T(0);
      }
    }
    if (GHOST) {
#pragma unroll
      for (int k = 0; k < S::GhostPer; ++k) {
        const int e = g0 + t + k * S::NT;
        gc[k] = -1;
        gv[k] = T(0);
        if (e < g1) {
          gc[k] = gcell[e];
          gv[k] = (T)gval[e];
        }
      }
    }
  }
  // LDS writes; the caller's barrier follows
  __device__ __forceinline__ void store(T* __restrict__ s, const int32_t* __restrict__ gcell,
                                        const double* __restrict__ gval) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < S::StagePer; ++r) {
      const int q = t + r * S::NT;
      if (q < kBoxOcts && (!GHOST || oq[r] >= 0)) {
        const int qx = q % 6, qy = (q / 6) % 6, qz = q / 36;
#pragma unroll
        for (int c = 0; c < 8; ++c)
          s[((2 * qz + (c >> 2)) * kBoxCells + 2 * qy + ((c >> 1) & 1)) * kBoxCells + 2 * qx + (c & 1)] = v[r][c];
      }
    }
    if (GHOST) {
#pragma unroll
      for (int k = 0; k < S::GhostPer; ++k)
        if (gc[k] >= 0) s[gc[k]] = gv[k];
      for (int e = g0 + t + S::GhostPer * S::NT; e < g1; e += S::NT) s[gcell[e]] = (T)gval[e];
    }
  }
};

// R consecutive values of an oct (p = oct base + c0, aligned to R values)
template <typename T, int R>
__device__ __forceinline__ void load_cells(const T* __restrict__ p, T (&v)[R]) {
  if constexpr (R * sizeof(T) >= 16) {
    using V = typename OctVec<T>::V;
    constexpr int VN = OctVec<T>::n;
#pragma unroll
    for (int k = 0; k < R / VN; ++k) {
      const V x = reinterpret_cast<const V*>(p)[k];
      const T* px = reinterpret_cast<const T*>(&x);
#pragma unroll
      for (int j = 0; j < VN; ++j) v[k * VN + j] = px[j];
    }
  } else {   // two floats
    const float2 x = *reinterpret_cast<const float2*>(p);
    v[0] = x.x;
    v[1] = x.y;
  }
}
template <typename T, int R>
__device__ __forceinline__ void store_cells(T* __restrict__ p, const T (&v)[R]) {
  if constexpr (R * sizeof(T) >= 16) {
    using V = typename OctVec<T>::V;
    constexpr int VN = OctVec<T>::n;
#pragma unroll
    for (int k = 0; k < R / VN; ++k) {
      V x;
      T* px = reinterpret_cast<T*>(&x);
#pragma unroll
      for (int j = 0; j < VN; ++j) px[j] = v[k * VN + j];
      reinterpret_cast<V*>(p)[k] = x;
    }
  } else {
    *reinterpret_cast<float2*>(p) = float2{v[0], v[1]};
  }
}

// Sum of the six neighbours of the thread's own cell k (box index i; k's low
// bits are the cell's cx and, for R = 4, cy): the neighbours inside the
// thread's cells from pv (registers), the rest from the box, added in the
// order -x, +x, -y, +y, -z, +z like a box-only sum.
template <typename T, int R>
__device__ __forceinline__ T own_nsum(const T* __restrict__ s, const T (&pv)[R], int k, int i) {
  const T xm = (k & 1) ? pv[k ^ 1] : s[i - 1];
  const T xp = (k & 1) ? s[i + 1] : pv[k ^ 1];
  T ym, yp;
  if constexpr (R >= 4) {
    ym = (k & 2) ? pv[k ^ 2] : s[i - kBoxCells];
    yp = (k & 2) ? s[i + kBoxCells] : pv[k ^ 2];
  } else {
    ym = s[i - kBoxCells];
    yp = s[i + kBoxCells];
  }
  return xm + xp + ym + yp + s[i - kBoxCells * kBoxCells] + s[i + kBoxCells * kBoxCells];
}
// box offset of cell c of an oct from the oct's cell 0
__device__ __forceinline__ constexpr int oct_cell_off(int c) {
  return (c & 1) + ((c >> 1) & 1) * kBoxCells + (c >> 2) * kBoxCells * kBoxCells;
}
// red cells: cx + cy + cz even
__device__ __forceinline__ constexpr bool cell_red(int c) { return (((c & 1) + ((c >> 1) & 1) + (c >> 2)) & 1) == 0; }

// box position of the brick's oct ob (0..63, x fastest), and of the oct holding box cell ci
__device__ __forceinline__ int brick_own_pos(int ob) {
  return (((ob >> 4) + 1) * 6 + ((ob >> 2) & 3) + 1) * 6 + (ob & 3) + 1;
}
// box index of cell 0 of the brick's oct ob
__device__ __forceinline__ int brick_oct_base(int ob) {
  return ((2 + 2 * (ob >> 4)) * kBoxCells + 2 + 2 * ((ob >> 2) & 3)) * kBoxCells + 2 + 2 * (ob & 3);
}
__device__ __forceinline__ int box_oct_of_cell(int ci) {
  const int x = ci % kBoxCells, y = (ci / kBoxCells) % kBoxCells, z = ci / (kBoxCells * kBoxCells);
  return ((z >> 1) * 6 + (y >> 1)) * 6 + (x >> 1);
}
__device__ __forceinline__ int cell_in_oct(int ci) {
  const int x = ci % kBoxCells, y = (ci / kBoxCells) % kBoxCells, z = ci / (kBoxCells * kBoxCells);
  return (x & 1) + 2 * (y & 1) + 4 * (z & 1);
}

// PROLONG: the sweep applies to src + P ec (trilinear prolongation of the
// coarse correction ec on the active cells of the box's octs): the brick's
// 8^3-cell coarse window (from the 5^3 coarse octs of cmap, shifted by the
// brick shift cshift) is staged in LDS first, and each box oct's correction
// is added as the oct is staged.
template <typename T, bool GHOST, bool ZERO, bool PROLONG, int R>
__global__ __launch_bounds__(BrickShape<R>::NT) __attribute__((amdgpu_waves_per_eu(R == 2 ? (PROLONG ? (GHOST ? 6 : 5) : 8) : (PROLONG ? 4 : 6)))) void k_brick_sweep(
    const int32_t* __restrict__ map, T h2, const T* __restrict__ src, const T* __restrict__ b, T* __restrict__ dst,
    const uint8_t* __restrict__ mask, const T* __restrict__ diag, const int32_t* __restrict__ gfirst,
    const int32_t* __restrict__ gcell, const double* __restrict__ gval, double* __restrict__ partials,
    const int32_t* __restrict__ cmap, int cshift, const T* __restrict__ ec, double* __restrict__ add64) {
  static_assert(!(GHOST && ZERO), "ghosts belong to the finest level, which never starts from zero");
  static_assert(!(PROLONG && ZERO), "a prolongation needs an incoming iterate");
  using S = BrickShape<R>;
  static_assert(S::NT >= kCoarseBoxOcts, "one coarse oct per thread");
  if constexpr (GHOST) {   // the finest level: every cell active, diagonal 6 (checked at launch)
    mask = nullptr;
    diag = nullptr;
  }
  __shared__ T s[kBoxCells * kBoxCells * kBoxCells];
  T* const sc = s;   // the 8^3 coarse window (prolongation), read before the box is staged over it
  const int t = threadIdx.x;
  const int ob = t / S::G, c0 = R * (t % S::G);   // own oct of the brick, own first cell
  const int64_t brick = xcd_block();   // neighbouring bricks share halo octs: keep them on one XCD
  const int32_t* bm = map + brick * kBoxOcts;
  // first batch of loads: map entries (box, own oct, the octs of this thread's red ring cells)
  BrickBox<T, ZERO, GHOST, R> box;
  box.load_map(bm, gfirst, brick);
  const int32_t own = bm[brick_own_pos(ob)];
  int sh_i[S::ShellPer];
  int32_t sh_o[S::ShellPer];
#pragma unroll
  for (int r = 0; r < S::ShellPer; ++r) {
    const int k = t + r * S::NT;
    sh_i[r] = kBrickShellCells.v[min(k, kBrickShell - 1)];
    sh_o[r] = k < kBrickShell ? bm[box_oct_of_cell(sh_i[r])] : -1;
  }
  int32_t co = -1;   // coarse oct t of the coarse box
  if (PROLONG && t < kCoarseBoxOcts) co = cmap[brick * kCoarseBoxOcts + t];
  // second batch: values
  box.load_values(src, gcell, gval);
  T cv[8];
  unsigned bmk[S::StagePer];   // active bits of the box octs (prolongation)
  if (PROLONG) {
    if (co >= 0) {
      load_oct(ec + (int64_t)co * 8, cv);
    } else {
#pragma unroll
      for (int c = 0; c < 8; ++c) cv[c] = T(0);
    }
#pragma unroll
    for (int r = 0; r < S::StagePer; ++r) bmk[r] = (mask && box.oq[r] >= 0) ? mask[box.oq[r]] : 0xFFu;
  }
  T bo[R], dg[R];   // b and the diagonal of the own cells
  unsigned mk = 0u;   // active bits of the own cells
  if (own >= 0) {
    mk = mask ? (unsigned)(mask[own] >> c0) & ((1u << R) - 1u) : (1u << R) - 1u;
    load_cells<T, R>(b + (int64_t)own * 8 + c0, bo);
    if (diag) {
      load_cells<T, R>(diag + (int64_t)own * 8 + c0, dg);
    } else {
#pragma unroll
      for (int k = 0; k < R; ++k) dg[k] = T(6);
    }
  }
  T sh_b[S::ShellPer], sh_d[S::ShellPer];   // b and (after the barrier) the inverse diagonal of the ring cells
  bool sh_on[S::ShellPer];
#pragma unroll
  for (int r = 0; r < S::ShellPer; ++r) {
    const int o = sh_o[r], c = cell_in_oct(sh_i[r]);
    sh_on[r] = o >= 0 && (!mask || ((mask[o] >> c) & 1u));
    sh_b[r] = T(0);
    sh_d[r] = T(1) / T(6);
    if (o >= 0) {
      sh_b[r] = b[(int64_t)o * 8 + c];
      if (diag) sh_d[r] = diag[(int64_t)o * 8 + c];
    }
  }
  if (PROLONG) {
    {
      // every window cell lies in exactly one coarse oct of the box: written
      // once, with the oct's value or 0 where the oct is absent
      const int sx = cshift & 1, sy = (cshift >> 1) & 1, sz = cshift >> 2;
      if (t < kCoarseBoxOcts) {
        const int ux = t % 5, uy = (t / 5) % 5, uz = t / 25;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int wx = 2 * ux + (c & 1) - sx, wy = 2 * uy + ((c >> 1) & 1) - sy, wz = 2 * uz + (c >> 2) - sz;
          if ((unsigned)wx < 8u && (unsigned)wy < 8u && (unsigned)wz < 8u) sc[(wz * 8 + wy) * 8 + wx] = cv[c];
        }
      }
    }
    __syncthreads();
    // box oct q = (qx, qy, qz) has its father at window cell (qx + 1, qy + 1, qz + 1)
#pragma unroll
    for (int r = 0; r < S::StagePer; ++r) {
      const int q = t + r * S::NT;
      if (q < kBoxOcts && box.oq[r] >= 0) {
        const int qx = q % 6, qy = (q / 6) % 6, qz = q / 36;
        // per axis 3/4 of the father and 1/4 of its neighbour on the child's side: z, then y, then x
        // (one cell plane at a time)
#pragma unroll
        for (int cz = 0; cz < 2; ++cz) {
          T zl[3][3];
#pragma unroll
          for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
              const int i = ((qz + 1) * 8 + qy + dy) * 8 + qx + dx;
              zl[dy][dx] = T(0.75) * sc[i] + T(0.25) * sc[cz ? i + 64 : i - 64];
            }
#pragma unroll
          for (int cy = 0; cy < 2; ++cy) {
            T yl[3];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) yl[dx] = T(0.75) * zl[1][dx] + T(0.25) * zl[2 * cy][dx];
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
              const int c = cx + 2 * cy + 4 * cz;
              if ((bmk[r] >> c) & 1u) box.v[r][c] += T(0.75) * yl[1] + T(0.25) * yl[2 * cx];
            }
          }
        }
      }
    }
  }
  if (PROLONG) __syncthreads();   // every correction has read the coarse window
  box.store(s, gcell, gval);
  __syncthreads();
  // inverse diagonals for the updates
  T idg[R];
#pragma unroll
  for (int k = 0; k < R; ++k) idg[k] = diag ? T(1) / dg[k] : T(1) / T(6);
  if (diag) {
#pragma unroll
    for (int r = 0; r < S::ShellPer; ++r) sh_d[r] = T(1) / sh_d[r];
  }

  auto nsum = [&](int i) {
    return s[i - 1] + s[i + 1] + s[i - kBoxCells] + s[i + kBoxCells] + s[i - kBoxCells * kBoxCells] +
           s[i + kBoxCells * kBoxCells];
  };
  const int i0 = brick_oct_base(ob) + oct_cell_off(c0);   // box index of the own cell k = 0
  // the own cells' values, kept in registers through both colours
  T pv[R];
#pragma unroll
  for (int k = 0; k < R; ++k) pv[k] = own >= 0 ? s[i0 + oct_cell_off(k)] : T(0);
  if (partials) {
    // ||b - L src||^2 over the brick's active cells, before any update
    // (uniform branch: `partials` is a kernel argument)
    double acc = 0.0;
    if (own >= 0) {
      const T inv_h2 = T(1) / h2;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if (!((mk >> k) & 1u)) continue;
        const T r = bo[k] - (own_nsum<T, R>(s, pv, k, i0 + oct_cell_off(k)) - dg[k] * pv[k]) * inv_h2;
        acc += (double)r * (double)r;
      }
    }
    const double tot = block_sum(acc);
    if (t == 0) partials[brick] = tot;
    __syncthreads();
  }
  // red: the brick's own cells and the ring
  if (own >= 0) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if (!cell_red(c0 + k) || !((mk >> k) & 1u)) continue;
      const int i = i0 + oct_cell_off(k);
      pv[k] = (own_nsum<T, R>(s, pv, k, i) - h2 * bo[k]) * idg[k];
      s[i] = pv[k];
    }
  }
#pragma unroll
  for (int r = 0; r < S::ShellPer; ++r)
    if (sh_on[r]) s[sh_i[r]] = (nsum(sh_i[r]) - h2 * sh_b[r]) * sh_d[r];
  __syncthreads();
  // black: the brick's own cells, then store them
  if (own >= 0) {
    T out[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int i = i0 + oct_cell_off(k);
      out[k] = (!cell_red(c0 + k) && ((mk >> k) & 1u)) ? (own_nsum<T, R>(s, pv, k, i) - h2 * bo[k]) * idg[k] : pv[k];
    }
    if (add64) {   // (uniform branch) the swept values are added to an f64 array instead
      double2* av = reinterpret_cast<double2*>(add64 + (int64_t)own * 8 + c0);
#pragma unroll
      for (int k = 0; k < R / 2; ++k) {
        double2 a = av[k];
        a.x += (double)out[2 * k];
        a.y += (double)out[2 * k + 1];
        av[k] = a;
      }
    } else {
      store_cells<T, R>(dst + (int64_t)own * 8 + c0, out);
    }
  }
}

// Residual on the brick's own octs from the staged box: r = b - (sum - diag e) / h^2
// on active cells (0 elsewhere); restricted to the father cell (bc[father],
// mean of the oct's 8, summed in cell order), and/or rounded to FP32 per cell
// (r32), and/or summed as ||r||^2 per brick (partials).
template <typename T, bool GHOST, int R>
__global__ __launch_bounds__(BrickShape<R>::NT) void k_brick_resid(const int32_t* __restrict__ map, T inv_h2,
                                                                   const T* __restrict__ e, const T* __restrict__ b,
                                                                   const uint8_t* __restrict__ mask,
                                                                   const T* __restrict__ diag,
                                                                   const int32_t* __restrict__ gfirst,
                                                                   const int32_t* __restrict__ gcell,
                                                                   const double* __restrict__ gval,
                                                                   const int32_t* __restrict__ father,
                                                                   T* __restrict__ bc, float* __restrict__ r32,
                                                                   double* __restrict__ partials) {
  using S = BrickShape<R>;
  if constexpr (GHOST) {   // the finest level: every cell active, diagonal 6 (checked at launch)
    mask = nullptr;
    diag = nullptr;
  }
  __shared__ T s[kBoxCells * kBoxCells * kBoxCells];
  const int t = threadIdx.x;
  const int sub = t % S::G, ob = t / S::G, c0 = R * sub;   // own oct of the brick, own first cell
  const int64_t brick = xcd_block();   // neighbouring bricks share halo octs: keep them on one XCD
  const int32_t* bm = map + brick * kBoxOcts;
  BrickBox<T, false, GHOST, R> box;
  box.load_map(bm, gfirst, brick);
  const int32_t own = bm[brick_own_pos(ob)];
  box.load_values(e, gcell, gval);
  T bo[R], dg[R];
  unsigned mk = 0u;
  int32_t fo = -1;
  if (own >= 0) {
    mk = mask ? (unsigned)(mask[own] >> c0) & ((1u << R) - 1u) : (1u << R) - 1u;
    load_cells<T, R>(b + (int64_t)own * 8 + c0, bo);
    if (diag) {
      load_cells<T, R>(diag + (int64_t)own * 8 + c0, dg);
    } else {
#pragma unroll
      for (int k = 0; k < R; ++k) dg[k] = T(6);
    }
    if (bc) fo = father[own];
  }
  box.store(s, gcell, gval);
  __syncthreads();
  double acc = 0.0;
  T rv[R];
#pragma unroll
  for (int k = 0; k < R; ++k) rv[k] = T(0);
  if (own >= 0) {
    const int i0 = brick_oct_base(ob) + oct_cell_off(c0);
    T pv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) pv[k] = s[i0 + oct_cell_off(k)];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if ((mk >> k) & 1u) rv[k] = bo[k] - (own_nsum<T, R>(s, pv, k, i0 + oct_cell_off(k)) - dg[k] * pv[k]) * inv_h2;
      acc += (double)rv[k] * (double)rv[k];
    }
    if (r32) {
      float* p = r32 + (int64_t)own * 8 + c0;
      if constexpr (R == 4) {
        *reinterpret_cast<float4*>(p) = float4{(float)rv[0], (float)rv[1], (float)rv[2], (float)rv[3]};
      } else {
        *reinterpret_cast<float2*>(p) = float2{(float)rv[0], (float)rv[1]};
      }
    }
  }
  if (bc) {   // (uniform branch) the oct's sum in cell order, passed along the oct's threads
    const int lead = (t & 63) - sub;   // lane of the oct's first thread
    T run = T(0);
#pragma unroll
    for (int j = 0; j < S::G; ++j) {
      if (sub == j) {
#pragma unroll
        for (int k = 0; k < R; ++k) run += rv[k];
      }
      run = __shfl(run, lead + j, 64);
    }
    if (sub == S::G - 1 && own >= 0 && fo >= 0) bc[fo] = run * T(0.125);
  }
  if (partials) {
    const double tot = block_sum(acc);
    if (t == 0) partials[brick] = tot;
  }
}

// coarsest oct level: red-black sweeps from a zero guess, all in LDS, one workgroup
constexpr int kCoarsestOcts = 256;
template <typename T>
__global__ __launch_bounds__(1024) void k_oct_coarsest(int n, T h2, T* __restrict__ e, const T* __restrict__ b,
                                                       const int32_t* __restrict__ nbr,
                                                       const uint8_t* __restrict__ mask,
                                                       const T* __restrict__ diag, int sweeps) {
  __shared__ T se[kCoarsestOcts * 8];
  __shared__ T sb[kCoarsestOcts * 8];
  __shared__ T sid[kCoarsestOcts * 8];
  __shared__ int32_t snb[kCoarsestOcts * 6];
  __shared__ uint8_t smk[kCoarsestOcts];
  for (int i = threadIdx.x; i < n * 8; i += blockDim.x) {
    se[i] = T(0);
    sb[i] = b[i];
    sid[i] = diag ? T(1) / diag[i] : T(1) / T(6);
  }
  for (int i = threadIdx.x; i < n * 6; i += blockDim.x) snb[i] = nbr[i];
  for (int i = threadIdx.x; i < n; i += blockDim.x) smk[i] = mask ? mask[i] : (uint8_t)0xFF;
  __syncthreads();
  for (int it = 0; it < sweeps; ++it) {
    for (int colour = 0; colour < 2; ++colour) {
      for (int i = threadIdx.x; i < n * 8; i += blockDim.x) {
        const int o = i >> 3, c = i & 7;
        if (((c ^ (c >> 1) ^ (c >> 2)) & 1) != colour || !((smk[o] >> c) & 1)) continue;
        T s = se[o * 8 + (c ^ 1)] + se[o * 8 + (c ^ 2)] + se[o * 8 + (c ^ 4)];
        for (int d = 0; d < 3; ++d) {
          const int v = snb[o * 6 + 2 * d + ((c >> d) & 1)];
          if (v >= 0) s += se[v * 8 + (c ^ (1 << d))];
        }
        se[i] = (s - h2 * sb[i]) * sid[i];
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n * 8; i += blockDim.x) e[i] = se[i];
}

// The tail V-cycle in one workgroup (see oct_tail): the same sweeps,
// residual + restriction and prolongation as the brick kernels, on compact
// lists of active cells, with e, b and every table in LDS.
constexpr int kTailThreads = 1024;
constexpr size_t kTailLdsBytes = 150 * 1024;
template <typename T>
__device__ __forceinline__ T tail_nsum(const T* __restrict__ se, const int16_t* __restrict__ nb, int i) {
  T v[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int q = nb[i * 6 + j];
    v[j] = q >= 0 ? se[q] : T(0);
  }
  return v[0] + v[1] + v[2] + v[3] + v[4] + v[5];
}
template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_oct_tail(TailArgs a, const uint4* __restrict__ blob,
                                                           const T* __restrict__ bt,
                                                           const int32_t* __restrict__ cell0, T* __restrict__ e0) {
  extern __shared__ __attribute__((aligned(16))) unsigned char tail_lds_base[];
  const int t = threadIdx.x;
  const int n = a.off[a.levels], nf = a.off[1];
  T* __restrict__ se = reinterpret_cast<T*>(tail_lds_base);
  T* __restrict__ sb = se + a.ns;
  // the table blob, laid out as in LDS: dg [n], nb [n][6], kids [n - nf][8], par [off[last]][8]
  uint4* lb = reinterpret_cast<uint4*>(sb + a.ns);
  const T* __restrict__ sdg = reinterpret_cast<const T*>(lb);
  const int16_t* __restrict__ snb = reinterpret_cast<const int16_t*>(sdg + n);
  const int16_t* __restrict__ skids = snb + 6 * n;
  const int16_t* __restrict__ spar = skids + 8 * (n - nf);
  // stage: every load of a pass in flight before its stores
  for (int base = 0; base < a.blob16; base += 4 * kTailThreads) {
    uint4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = base + u * kTailThreads + t;
      if (q < a.blob16) v[u] = blob[q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = base + u * kTailThreads + t;
      if (q < a.blob16) lb[q] = v[u];
    }
  }
  for (int i = t; i < nf; i += kTailThreads) sb[i] = bt[i];
  __syncthreads();
  auto sweeps = [&](int k, int count) {
    const T h2 = (T)a.h2[k];
    for (int it = 0; it < count; ++it) {
      for (int colour = 0; colour < 2; ++colour) {
        const int lo = colour ? a.off[k] + a.nred[k] : a.off[k];
        const int hi = colour ? a.off[k + 1] : a.off[k] + a.nred[k];
        for (int i = lo + t; i < hi; i += kTailThreads)
          se[i] = (tail_nsum(se, snb, i) - h2 * sb[i]) * (T(1) / sdg[i]);
        __syncthreads();
      }
    }
  };
  auto zero = [&](int k) {
    for (int i = a.off[k] + t; i < a.off[k + 1]; i += kTailThreads) se[i] = T(0);
    __syncthreads();
  };
  // down: pre-smoothing from zero, residual restricted to the next level
  for (int k = 0; k + 1 < a.levels; ++k) {
    zero(k);
    sweeps(k, a.nu_pre);
    const T inv_h2 = (T)a.inv_h2[k];
    for (int F = a.off[k + 1] + t; F < a.off[k + 2]; F += kTailThreads) {
      T rsum = T(0);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int q = skids[(F - nf) * 8 + c];
        T r = T(0);
        if (q >= 0) r = sb[q] - (tail_nsum(se, snb, q) - sdg[q] * se[q]) * inv_h2;
        rsum += r;
      }
      sb[F] = rsum * T(0.125);
    }
    __syncthreads();
  }
  zero(a.levels - 1);
  sweeps(a.levels - 1, a.last_sweeps);
  // up: prolongation + correction, post-smoothing
  for (int k = a.levels - 2; k >= 0; --k) {
    for (int i = a.off[k] + t; i < a.off[k + 1]; i += kTailThreads) {
      T E[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int q = spar[i * 8 + j];
        E[j] = q >= 0 ? se[q] : T(0);
      }
      const T z00 = T(0.75) * E[0] + T(0.25) * E[1], z01 = T(0.75) * E[2] + T(0.25) * E[3];
      const T z10 = T(0.75) * E[4] + T(0.25) * E[5], z11 = T(0.75) * E[6] + T(0.25) * E[7];
      const T y0 = T(0.75) * z00 + T(0.25) * z01, y1 = T(0.75) * z10 + T(0.25) * z11;
      se[i] += T(0.75) * y0 + T(0.25) * y1;
    }
    __syncthreads();
    sweeps(k, a.nu_post);
  }
  for (int i = t; i < nf; i += kTailThreads) e0[cell0[i]] = se[i];
}

__global__ __launch_bounds__(kBlock) void k_ghost_values(int64_t n_ghost, const int32_t* __restrict__ gidx,
                                                         const double* __restrict__ phi_parent,
                                                         double* __restrict__ gval) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (ghost face, cell) pair
  if (t >= n_ghost * 4) return;
  const int32_t* id = gidx + t * 8;
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int a = (q >> 2) & 1, b = (q >> 1) & 1, c = q & 1;
    const double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
    v += w * phi_parent[id[q]];
  }
  gval[t] = v;
}

// Squared norm, per workgroup, of the level's full right-hand side
// b = f - (sum of the ghost neighbours) / h^2: the residual of the zero
// potential, the scale the refined level's relative residual is taken on.
__global__ __launch_bounds__(kBlock) void k_oct_rhs_norm(int64_t n, double inv_h2, const double* __restrict__ f,
                                                         const int32_t* __restrict__ nbr,
                                                         const double* __restrict__ ghost,
                                                         double* __restrict__ partials) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (o < n) {
    int32_t nb[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) nb[j] = nbr[o * 6 + j];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      double g = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int v = nb[2 * d + ((c >> d) & 1)];
        if (v <= -2) g += ghost[(int64_t)(-2 - v) * 4 + face_slot(c, d)];
      }
      const double b = f[o * 8 + c] - g * inv_h2;
      acc += b * b;
    }
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void morton_keys(int64_t n, const int32_t* ijk, uint64_t* keys, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_morton, dim3(grid_for(n)), dim3(kBlock), 0, s, n, ijk, keys);
  check_launch();
}

void oct_validate(int64_t n, const int32_t* ijk, int n_dim, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(grid_for(n)), dim3(kBlock), 0, s, n, ijk, n_dim, flag);
  check_launch();
}

size_t hash_slot_bytes() { return sizeof(Slot); }

void hash_build(int64_t n, const uint64_t* keys, void* table, int64_t cap, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_hash_clear, dim3(grid_for(cap)), dim3(kBlock), 0, s, cap, (Slot*)table);
  if (n > 0)
    hipLaunchKernelGGL(k_hash_insert, dim3(grid_for(n)), dim3(kBlock), 0, s, n, keys, (Slot*)table,
                       (uint64_t)(cap - 1), flag);
  check_launch();
}

void hash_lookup_many(int64_t n, const uint64_t* q, const void* table, int64_t cap, int32_t* out, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_hash_lookup, dim3(grid_for(n)), dim3(kBlock), 0, s, n, q, (const Slot*)table,
                     (uint64_t)(cap - 1), out);
  check_launch();
}

void nbr_from_hash(int64_t n, const uint64_t* keys, int n_dim, const void* table, int64_t cap, int32_t* nbr,
                   int32_t* missing, hipStream_t s) {
  hipLaunchKernelGGL(k_nbr_hash, dim3(grid_for(n * 8)), dim3(kBlock), 0, s, n, keys, n_dim, (const Slot*)table,
                     (uint64_t)(cap - 1), nbr, missing);
  check_launch();
}

void exclusive_scan_i32(int64_t n, const int32_t* in, int32_t* out, hipStream_t s) {
  size_t tb = 0;
  MG_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, in, out, (int)n, s));
  DevBuf tmp;
  tmp.scratch(tb > 0 ? tb : 1, s);
  MG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tb, in, out, (int)n, s));
}

void ghost_stencils(int64_t n, const uint64_t* keys, int n_dim, const int32_t* first, int32_t* nbr,
                    bool parent_uniform, const void* ptable, int64_t pcap, int pcells, const int (&shift)[3],
                    int32_t* gidx, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_ghost_stencil, dim3(grid_for(n * 8)), dim3(kBlock), 0, s, n, keys, n_dim, first, nbr,
                     parent_uniform ? 1 : 0, (const Slot*)ptable, (uint64_t)(pcap > 0 ? pcap - 1 : 0), pcells,
                     shift[0], shift[1], shift[2], gidx, flag);
  check_launch();
}

__global__ __launch_bounds__(kBlock) void k_brick_ghost_pack(int64_t n, const int32_t* __restrict__ gidx,
                                                             const double* __restrict__ gval,
                                                             double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = gval[gidx[i]];
}

void brick_ghost_pack(int64_t n, const int32_t* gidx, const double* gval, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_brick_ghost_pack, dim3(grid_for(n)), dim3(kBlock), 0, s, n, gidx, gval, out);
  check_launch();
}

int64_t oct_rhs_norm2(int64_t n, double h, const double* f, const int32_t* nbr, const double* ghost, double* partials,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_oct_rhs_norm, dim3(grid_for(n)), dim3(kBlock), 0, s, n, 1.0 / (h * h), f, nbr, ghost, partials);
  check_launch();
  return grid_for(n);
}

void ghost_values(int64_t n_ghost, const int32_t* gidx, const double* phi_parent, double* gval, hipStream_t s) {
  if (n_ghost == 0) return;
  hipLaunchKernelGGL(k_ghost_values, dim3(grid_for(n_ghost * 4)), dim3(kBlock), 0, s, n_ghost, gidx, phi_parent,
                     gval);
  check_launch();
}

// Sorted unique ancestor keys (key >> drop: parents for drop 3) of `keys`;
// returns the count (synchronises).  Keys already in ascending order
// (`sorted`) have their ancestors in ascending order too, and skip the sort
// (key_bits: significant bits of the ancestor keys).  `out` is allocated, with
// room for n keys, as scratch on s (out_scratch) or as a level buffer.
int64_t unique_parent_keys(int64_t n, const uint64_t* keys, DevBuf& out, int key_bits, bool sorted,
                           bool out_scratch, hipStream_t s, int drop) {
  DevBuf pk, srt, cnt;
  pk.scratch(n * sizeof(uint64_t), s);
  if (!sorted) srt.scratch(n * sizeof(uint64_t), s);
  cnt.scratch(sizeof(int32_t), s);
  hipLaunchKernelGGL(k_parent_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, n, keys, drop, pk.as<uint64_t>());
  check_launch();
  // unique from `in` straight into out (room for n keys)
  const uint64_t* in = sorted ? pk.as<uint64_t>() : srt.as<uint64_t>();
  if (out_scratch) out.scratch(std::max<int64_t>(n, 1) * sizeof(uint64_t), s);
  else out.alloc(std::max<int64_t>(n, 1) * sizeof(uint64_t));
  size_t tb = 0, tb2 = 0;
  if (!sorted)
    MG_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, pk.as<uint64_t>(), srt.as<uint64_t>(), (int)n, 0,
                                             key_bits, s));
  MG_HIP(hipcub::DeviceSelect::Unique(nullptr, tb2, in, out.as<uint64_t>(), cnt.as<int32_t>(), (int)n, s));
  DevBuf tmp;
  tmp.scratch(std::max<size_t>(std::max(tb, tb2), 1), s);
  if (!sorted)
    MG_HIP(hipcub::DeviceRadixSort::SortKeys(tmp.p, tb, pk.as<uint64_t>(), srt.as<uint64_t>(), (int)n, 0,
                                             key_bits, s));
  MG_HIP(hipcub::DeviceSelect::Unique(tmp.p, tb2, in, out.as<uint64_t>(), cnt.as<int32_t>(), (int)n, s));
  int32_t count = 0;
  MG_HIP(hipMemcpyAsync(&count, cnt.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  return count;
}

// *count += set bits of mask[0..n) (active cells of a coarse level)
__global__ __launch_bounds__(kBlock) void k_count_active(int64_t n, const uint8_t* __restrict__ mask,
                                                          unsigned long long* __restrict__ count) {
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += (unsigned long long)__popc((unsigned)mask[i]);
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

void count_active(int64_t n, const uint8_t* mask, unsigned long long* count, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_count_active, dim3(g), dim3(kBlock), 0, s, n, mask, count);
  check_launch();
}

void fathers(int64_t n, const uint64_t* keys, const uint64_t* ckeys, int64_t nc, int32_t* father, int* flag,
             hipStream_t s) {
  hipLaunchKernelGGL(k_fathers, dim3(grid_for(n)), dim3(kBlock), 0, s, n, keys, ckeys, nc, father, flag);
  check_launch();
}

void coarse_level_set(int64_t n_fine, const int32_t* father, const float* fine_lsm, int64_t n_coarse,
                      float* coarse_lsm, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n_coarse * 8)), dim3(kBlock), 0, s, n_coarse * 8, -1.0f, coarse_lsm);
  hipLaunchKernelGGL(k_coarse_lsm, dim3(grid_for(n_fine)), dim3(kBlock), 0, s, n_fine, father, fine_lsm, coarse_lsm);
  check_launch();
}

template <typename T>
void level_set_operator(int64_t n, const int32_t* nbr, const float* lsm, uint8_t* mask, T* diag, hipStream_t s) {
  hipLaunchKernelGGL((k_lsm_operator<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, nbr, lsm, mask, diag);
  check_launch();
}
template void level_set_operator<double>(int64_t, const int32_t*, const float*, uint8_t*, double*, hipStream_t);
template void level_set_operator<float>(int64_t, const int32_t*, const float*, uint8_t*, float*, hipStream_t);

void nbr_sorted(int64_t n, const uint64_t* keys, int n_dim, int32_t* nbr, int32_t* nbr27, hipStream_t s) {
  MG_REQUIRE(nbr != nullptr && nbr27 != nullptr, "internal: nbr_sorted fills both tables");
  hipLaunchKernelGGL(k_nbr_sorted, dim3(grid_for(n * 27)), dim3(kBlock), 0, s, n, keys, n_dim, nbr, nbr27);
  check_launch();
}

template <typename T>
void oct_smooth(int64_t n, double h, T* e, const T* b, const int32_t* nbr, const uint8_t* mask,
                const T* diag, const double* ghost, int sweeps, hipStream_t s) {
  const T h2 = (T)(h * h);
  for (int it = 0; it < sweeps; ++it) {
    if (ghost) {
      hipLaunchKernelGGL((k_oct_smooth<T, 0, true>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, h2, e, b, nbr, mask, diag, ghost);
      hipLaunchKernelGGL((k_oct_smooth<T, 1, true>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, h2, e, b, nbr, mask, diag, ghost);
    } else {
      hipLaunchKernelGGL((k_oct_smooth<T, 0, false>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, h2, e, b, nbr, mask, diag, ghost);
      hipLaunchKernelGGL((k_oct_smooth<T, 1, false>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, h2, e, b, nbr, mask, diag, ghost);
    }
  }
  check_launch();
}

template <typename T>
void oct_resid(int64_t n, double h, const T* e, const T* b, const int32_t* nbr, const uint8_t* mask,
               const T* diag, const double* ghost, const int32_t* father, T* bc, float* r32,
               double* partials, hipStream_t s) {
  const T inv_h2 = (T)(1.0 / (h * h));
  const dim3 g(grid_for(n)), bl(kBlock);
  if (ghost) {
    if (bc) hipLaunchKernelGGL((k_oct_resid<T, true, true>), g, bl, 0, s, n, inv_h2, e, b, nbr, mask, diag, ghost, father, bc, r32, partials);
    else hipLaunchKernelGGL((k_oct_resid<T, true, false>), g, bl, 0, s, n, inv_h2, e, b, nbr, mask, diag, ghost, father, bc, r32, partials);
  } else {
    if (bc) hipLaunchKernelGGL((k_oct_resid<T, false, true>), g, bl, 0, s, n, inv_h2, e, b, nbr, mask, diag, ghost, father, bc, r32, partials);
    else hipLaunchKernelGGL((k_oct_resid<T, false, false>), g, bl, 0, s, n, inv_h2, e, b, nbr, mask, diag, ghost, father, bc, r32, partials);
  }
  check_launch();
}


template <typename T>
void oct_prolong(int64_t n, const int32_t* father, const int32_t* cnbr27, const T* ec, T* e, const uint8_t* mask,
                 hipStream_t s) {
  hipLaunchKernelGGL((k_oct_prolong<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, father, cnbr27, ec, e, mask);
  check_launch();
}

int64_t brick_keys(int64_t n, const uint64_t* keys, bool sorted, int n_dim, int shift, DevBuf& out,
                   hipStream_t s) {
  const int bits = std::min(64, 3 * std::max(1, ilog2(n_dim)));
  DevBuf shifted;
  if (shift != 0) {
    shifted.scratch(n * sizeof(uint64_t), s);
    sorted = false;
    hipLaunchKernelGGL(k_shift_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, n, keys, n_dim, shift,
                       shifted.as<uint64_t>());
    check_launch();
    keys = shifted.as<uint64_t>();
  }
  // brick keys: the (shifted) keys' ancestors two levels up
  return unique_parent_keys(n, keys, out, std::max(3, bits - 6), sorted, true, s, 6);
}

int choose_brick_shift(int64_t n, const uint64_t* keys, int n_dim, hipStream_t s) {
  // one bit per brick of each of the 8 lattices: (n_dim / 4)^3 bits each
  if (n < kBrickShiftMinOcts || n_dim < 8 || n_dim > kBrickShiftMaxDim) return 0;
  const int64_t nb = n_dim / 4;
  const int64_t words_per = (nb * nb * nb + 31) / 32;
  DevBuf bits, counts;
  bits.scratch(8 * words_per * sizeof(uint32_t), s);
  counts.scratch(8 * sizeof(unsigned long long), s);
  MG_HIP(hipMemsetAsync(bits.p, 0, 8 * words_per * sizeof(uint32_t), s));
  MG_HIP(hipMemsetAsync(counts.p, 0, 8 * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_brick_shift_bits, dim3(grid_for(n)), dim3(kBlock), 0, s, n, keys, n_dim, words_per,
                     bits.as<uint32_t>());
  const unsigned gx = (unsigned)std::min<int64_t>(256, (words_per + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_brick_shift_count, dim3(gx, 8), dim3(kBlock), 0, s, words_per, bits.as<uint32_t>(),
                     counts.as<unsigned long long>());
  check_launch();
  unsigned long long c[8];
  MG_HIP(hipMemcpyAsync(c, counts.p, sizeof(c), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  int best = 0;
  for (int j = 1; j < 8; ++j)
    if (c[j] < c[best]) best = j;   // ties keep the smaller shift, the aligned lattice first
  return best;
}

void brick_map(int64_t n_bricks, const uint64_t* bkeys, int n_dim, int shift, const void* table, int64_t cap,
               const uint64_t* sorted_keys, int64_t n_sorted, int32_t* map, hipStream_t s) {
  const int64_t items = n_bricks * kBoxOcts;
  hipLaunchKernelGGL(k_brick_map, dim3(grid_for(items)), dim3(kBlock), 0, s, n_bricks, bkeys, n_dim, shift,
                     static_cast<const Slot*>(table), (uint64_t)(cap - 1), sorted_keys, n_sorted, map);
  check_launch();
}

void brick_cmap(int64_t n_bricks, const uint64_t* bkeys, int n_dim_c, int shift, const uint64_t* ckeys,
                int64_t n_coarse, int32_t* cmap, hipStream_t s) {
  const int64_t items = n_bricks * kCoarseBoxOcts;
  hipLaunchKernelGGL(k_brick_cmap, dim3(grid_for(items)), dim3(kBlock), 0, s, n_bricks, bkeys, n_dim_c, shift,
                     ckeys, n_coarse, cmap);
  check_launch();
}

int64_t brick_ghosts(int64_t n_bricks, const int32_t* map, const int32_t* nbr, DevBuf& first, DevBuf& cell,
                     DevBuf& gv, hipStream_t s) {
  const int64_t items = n_bricks * kBoxOcts;
  DevBuf count;
  count.scratch(items * sizeof(int32_t), s);
  first.alloc((items + 1) * sizeof(int32_t));
  hipLaunchKernelGGL(k_brick_ghost_count, dim3(grid_for(items)), dim3(kBlock), 0, s, n_bricks, map, nbr,
                     count.as<int32_t>());
  check_launch();
  exclusive_scan_i32(items, count.as<int32_t>(), first.as<int32_t>(), s);
  int32_t last[2] = {0, 0};
  MG_HIP(hipMemcpyAsync(&last[0], first.as<int32_t>() + (items - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MG_HIP(hipMemcpyAsync(&last[1], count.as<int32_t>() + (items - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  const int64_t total = (int64_t)last[0] + last[1];
  const int32_t total32 = (int32_t)total;
  MG_HIP(hipMemcpyAsync(first.as<int32_t>() + items, &total32, sizeof(int32_t), hipMemcpyHostToDevice, s));
  cell.alloc(std::max<int64_t>(total, 1) * sizeof(int32_t));
  gv.alloc(std::max<int64_t>(total, 1) * sizeof(int32_t));
  hipLaunchKernelGGL(k_brick_ghost_fill, dim3(grid_for(items)), dim3(kBlock), 0, s, n_bricks, map, nbr,
                     first.as<int32_t>(), cell.as<int32_t>(), gv.as<int32_t>());
  check_launch();
  MG_HIP(hipStreamSynchronize(s));
  return total;
}

template <typename T>
void brick_sweep(int64_t n_bricks, const int32_t* map, double h, const T* src, const T* b, T* dst,
                 const uint8_t* mask, const T* diag, const BrickGhosts& gh, hipStream_t s, double* partials,
                 const int32_t* cmap, int cshift, const T* ec, double* add64) {
  MG_REQUIRE(!(gh.val && src == nullptr), "internal: a zero-guess brick sweep has no ghosts");
  MG_REQUIRE(!(ec && (src == nullptr || cmap == nullptr)), "internal: a prolongation needs src and the coarse map");
  MG_REQUIRE(!(gh.val && (mask || diag)), "internal: a level with ghosts has all cells active and diagonal 6");
  const T h2 = (T)(h * h);
  const dim3 grid((unsigned)n_bricks);
#define MG_BRICK_SWEEP(G, Z, P)                                                                                   \
  hipLaunchKernelGGL((k_brick_sweep<T, G, Z, P, P ? kProlongCells : kSweepCells<T>>), grid,                       \
                     dim3(BrickShape<P ? kProlongCells : kSweepCells<T>>::NT), 0, s, map, h2, src, b, dst, mask, diag, \
                     gh.first, gh.cell, gh.val, partials, cmap, cshift, ec, add64)
  if (gh.val && ec) MG_BRICK_SWEEP(true, false, true);
  else if (gh.val) MG_BRICK_SWEEP(true, false, false);
  else if (ec) MG_BRICK_SWEEP(false, false, true);
  else if (src == nullptr) MG_BRICK_SWEEP(false, true, false);
  else MG_BRICK_SWEEP(false, false, false);
#undef MG_BRICK_SWEEP
  check_launch();
}
template void brick_sweep<double>(int64_t, const int32_t*, double, const double*, const double*, double*,
                                  const uint8_t*, const double*, const BrickGhosts&, hipStream_t, double*,
                                  const int32_t*, int, const double*, double*);
template void brick_sweep<float>(int64_t, const int32_t*, double, const float*, const float*, float*,
                                 const uint8_t*, const float*, const BrickGhosts&, hipStream_t, double*,
                                 const int32_t*, int, const float*, double*);

template <typename T>
void brick_resid(int64_t n_bricks, const int32_t* map, double h, const T* e, const T* b, const uint8_t* mask,
                 const T* diag, const BrickGhosts& gh, const int32_t* father, T* bc, float* r32, double* partials,
                 hipStream_t s) {
  const T inv_h2 = (T)(1.0 / (h * h));
  const dim3 grid((unsigned)n_bricks), block(BrickShape<kResidCells>::NT);
  MG_REQUIRE(!(gh.val && (mask || diag)), "internal: a level with ghosts has all cells active and diagonal 6");
  if (gh.val)
    hipLaunchKernelGGL((k_brick_resid<T, true, kResidCells>), grid, block, 0, s, map, inv_h2, e, b, mask, diag, gh.first, gh.cell,
                       gh.val, father, bc, r32, partials);
  else
    hipLaunchKernelGGL((k_brick_resid<T, false, kResidCells>), grid, block, 0, s, map, inv_h2, e, b, mask, diag, gh.first, gh.cell,
                       gh.val, father, bc, r32, partials);
  check_launch();
}
template void brick_resid<double>(int64_t, const int32_t*, double, const double*, const double*, const uint8_t*,
                                  const double*, const BrickGhosts&, const int32_t*, double*, float*, double*,
                                  hipStream_t);
template void brick_resid<float>(int64_t, const int32_t*, double, const float*, const float*, const uint8_t*,
                                 const float*, const BrickGhosts&, const int32_t*, float*, float*, double*,
                                 hipStream_t);

int coarsest_oct_capacity() { return kCoarsestOcts; }

void oct_force(int64_t n, double h, const double* phi, const int32_t* nbr, const double* ghost, double* g,
               hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_oct_force, dim3(grid_for(4 * n)), dim3(kBlock), 0, s, n, 0.5 / h, phi, nbr, ghost, g);
  check_launch();
}

void nbr_export(int64_t n, const int32_t* nbr, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_nbr_export, dim3(grid_for(n * 6)), dim3(kBlock), 0, s, n * 6, nbr, out);
  check_launch();
}

size_t tail_blob_bytes(int64_t n, int64_t n_first, int64_t n_last, size_t elem_bytes) {
  const size_t b = (size_t)n * (elem_bytes + 12) + (size_t)(n - n_first) * 16 + (size_t)(n - n_last) * 16;
  return (b + 15) / 16 * 16;
}
size_t tail_lds_bytes(int64_t n, int64_t n_first, int64_t n_last, size_t elem_bytes) {
  return 2 * (size_t)((n + 3) / 4 * 4) * elem_bytes + tail_blob_bytes(n, n_first, n_last, elem_bytes);
}
size_t tail_lds_limit() { return kTailLdsBytes; }

template <typename T>
void oct_tail(const TailArgs& a, const void* blob, const T* bt, const int32_t* cell0, T* e0, hipStream_t s) {
  const int n = a.off[a.levels];
  const size_t lds = tail_lds_bytes(n, a.off[1], n - a.off[a.levels - 1], sizeof(T));
  MG_REQUIRE(a.levels >= 1 && a.levels <= kTailMaxLevels && lds <= kTailLdsBytes && a.ns == (n + 3) / 4 * 4 &&
                 (size_t)a.blob16 * 16 == tail_blob_bytes(n, a.off[1], n - a.off[a.levels - 1], sizeof(T)),
             "internal: tail layout");
  static bool attr_set = false;   // per template instance, for the largest size the tail may take
  if (!attr_set) {
    MG_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_oct_tail<T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTailLdsBytes));
    attr_set = true;
  }
  hipLaunchKernelGGL((k_oct_tail<T>), dim3(1), dim3(kTailThreads), lds, s, a, static_cast<const uint4*>(blob), bt,
                     cell0, e0);
  check_launch();
}
template void oct_tail<double>(const TailArgs&, const void*, const double*, const int32_t*, double*, hipStream_t);
template void oct_tail<float>(const TailArgs&, const void*, const float*, const int32_t*, float*, hipStream_t);

template <typename T>
void oct_coarsest(int64_t n, double h, T* e, const T* b, const int32_t* nbr, const uint8_t* mask,
                  const T* diag, int sweeps, hipStream_t s) {
  hipLaunchKernelGGL((k_oct_coarsest<T>), dim3(1), dim3(1024), 0, s, (int)n, (T)(h * h), e, b, nbr, mask, diag,
                     sweeps);
  check_launch();
}

#define MG_INST(T)                                                                                              \
  template void oct_smooth<T>(int64_t, double, T*, const T*, const int32_t*, const uint8_t*, const T*,           \
                              const double*, int, hipStream_t);                                                 \
  template void oct_resid<T>(int64_t, double, const T*, const T*, const int32_t*, const uint8_t*, const T*,        \
                             const double*, const int32_t*, T*, float*, double*, hipStream_t);                  \
  template void oct_prolong<T>(int64_t, const int32_t*, const int32_t*, const T*, T*, const uint8_t*, hipStream_t); \
  template void oct_coarsest<T>(int64_t, double, T*, const T*, const int32_t*, const uint8_t*, const T*, int,       \
                                hipStream_t);
MG_INST(double)
MG_INST(float)
#undef MG_INST

}  // namespace mg

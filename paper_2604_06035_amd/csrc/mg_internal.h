// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mg.h"

namespace mg {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* get_error();

struct Fail {
  mg_status_t status;
};

#define MG_HIP(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ::mg::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));               \
      throw ::mg::Fail{e_ == hipErrorOutOfMemory ? MG_ERR_OOM : MG_ERR_HIP};            \
    }                                                                                   \
  } while (0)

#define MG_REQUIRE(cond, msg)                                                           \
  do {                                                                                  \
    if (!(cond)) {                                                                      \
      ::mg::set_error(msg);                                                             \
      throw ::mg::Fail{MG_ERR_ARG};                                                     \
    }                                                                                   \
  } while (0)

inline void check_launch() { MG_HIP(hipGetLastError()); }

// every extern "C" entry point body: C++ failures become a status, never an exception
#define MG_API_BEGIN try {
#define MG_API_END                                      \
  }                                                     \
  catch (const ::mg::Fail& f) {                         \
    return f.status;                                    \
  }                                                     \
  catch (const std::bad_alloc&) {                       \
    ::mg::set_error("host allocation failed");          \
    return MG_ERR_OOM;                                  \
  }                                                     \
  catch (...) {                                         \
    ::mg::set_error("unexpected C++ exception");        \
    return MG_ERR_HIP;                                  \
  }

// ---------------------------------------------------------------------------
// device buffers owned by a handle
// ---------------------------------------------------------------------------
// A level build makes a hundred or more allocations, many of them small:
// while a DevArena is installed on the building thread (ArenaScope), DevBuf
// allocations are carved from the arena's large chunks (freed with the
// arena, not one by one), and a build step's scratch buffers come from the
// device's stream-ordered pool on the build stream (DevBuf::scratch).
struct DevArena {
  static constexpr size_t kChunk = size_t(64) << 20;   // chunk size
  static constexpr size_t kAlone = size_t(8) << 20;    // requests from here up get their own allocation
  static constexpr size_t kAlign = 256;
  struct Block {
    void* p;
    size_t bytes;
  };
  std::vector<Block> blocks;
  int device = -1;
  char* cur = nullptr;
  size_t left = 0;
  DevArena() = default;
  DevArena(const DevArena&) = delete;
  DevArena& operator=(const DevArena&) = delete;
  ~DevArena() { release(); }
  void* get(size_t b);
  // waits for the device, then hands the blocks to the device's block cache
  void release() noexcept;
};
// the arenas that DevBuf::alloc and DevBuf::scratch draw from on this thread
// (null: hipMalloc, and the stream-ordered pool)
DevArena*& current_arena();
DevArena*& current_scratch_arena();
struct ArenaScope {
  DevArena* prev;
  DevArena* prev_scratch;
  // a: the level's buffers; scr: the build's scratch (released by its owner
  // once the build's work is done)
  ArenaScope(DevArena* a, DevArena* scr) : prev(current_arena()), prev_scratch(current_scratch_arena()) {
    current_arena() = a;
    current_scratch_arena() = scr;
  }
  ~ArenaScope() {
    current_arena() = prev;
    current_scratch_arena() = prev_scratch;
  }
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;
};
// the device's stream-ordered pool, set (once per device) to keep freed
// memory for reuse instead of returning it at every synchronisation
void prepare_scratch_pool();

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = false;    // p is freed by this buffer (not part of an arena)
  bool pooled = false;   // p came from the stream-ordered pool on `ps`
  hipStream_t ps = nullptr;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned), pooled(o.pooled), ps(o.ps) { o.forget(); }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      owned = o.owned;
      pooled = o.pooled;
      ps = o.ps;
      o.forget();
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    if (DevArena* a = current_arena()) {
      p = a->get(b);
    } else {
      MG_HIP(hipMalloc(&p, b));
      owned = true;
    }
    bytes = b;
  }
  // scratch of one step on stream s: from the build's scratch arena if one is
  // installed, else from the stream-ordered pool, returned to it (in stream
  // order) when the buffer is released; s must outlive the buffer
  void scratch(size_t b, hipStream_t s) {
    release();
    if (b == 0) return;
    if (DevArena* a = current_scratch_arena()) {
      p = a->get(b);
      bytes = b;
      return;
    }
    prepare_scratch_pool();
    MG_HIP(hipMallocAsync(&p, b, s));
    owned = pooled = true;
    ps = s;
    bytes = b;
  }
  void release() {
    if (p && owned) {
      if (pooled) (void)hipFreeAsync(p, ps);
      else (void)hipFree(p);
    }
    forget();
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }

 private:
  void forget() {
    p = nullptr;
    bytes = 0;
    owned = pooled = false;
    ps = nullptr;
  }
};

// ---------------------------------------------------------------------------
// Morton keys (equation morton_encode: bit b of x, y, z -> key bits 3b, 3b+1,
// 3b+2) by shift-and-mask bit spreading of 21-bit fields, and the table hash
// of equation hash_func on a 64-bit (reduced) key
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
__device__ __forceinline__ uint32_t compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v | (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v | (v >> 4)) & 0x100f00f00f00f00full;
  v = (v | (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v | (v >> 16)) & 0x1f00000000ffffull;
  v = (v | (v >> 32)) & 0x1fffffull;
  return (uint32_t)v;
}
__device__ __forceinline__ uint64_t morton(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}
__device__ __forceinline__ void unmorton(uint64_t k, int& x, int& y, int& z) {
  x = (int)compact3(k);
  y = (int)compact3(k >> 1);
  z = (int)compact3(k >> 2);
}

__device__ __forceinline__ uint64_t hash64(uint64_t k) {
  const uint64_t phi1 = 2654435761ull, phi2 = 0x9E3779B97F4A7C15ull;
  const uint64_t t = ((k * phi1) ^ (k >> 16)) * phi2;
  return t ^ (t >> 13);
}

// Workgroup index in XCD-contiguous order.  The hardware deals workgroups
// to the 8 XCDs in turn (workgroup b runs on XCD b % 8), each with its own
// L2; renumbering gives every XCD one contiguous run of the grid (XCD x takes
// G / 8 workgroups, one more when x < G % 8), so workgroups that read each
// other's neighbourhoods share an L2.
__device__ __forceinline__ unsigned xcd_block() {
  const unsigned b = blockIdx.x, G = gridDim.x;
  const unsigned q = G >> 3, r = G & 7u, x = b & 7u, i = b >> 3;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Store of a 16-byte pair with the nontemporal hint: for outputs written
// once and not read back by the same kernel (keeps them from displacing
// inputs that neighbouring workgroups still read from L2).
__device__ __forceinline__ void stream_store(double2* p, double2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

// Sum of v over the workgroup (any size up to 1024 threads, whole waves) in
// a fixed order; the result is valid in thread 0.  Contains a barrier, so
// every thread of the workgroup calls it; two calls need a barrier between
// them (the shared slots are reused).
__device__ __forceinline__ double block_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double ws[1024 / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) ws[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) t += ws[i];
  return t;
}

inline int ilog2(int64_t v) {
  int r = 0;
  while ((int64_t(1) << r) < v) ++r;
  return r;
}
inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// ---------------------------------------------------------------------------
// kernel launchers: full periodic grids (uniform.hip)
// ---------------------------------------------------------------------------
// Partial-sum scratch: every reduction writes one f64 per workgroup, then a
// single-workgroup kernel adds them in a fixed order (deterministic).
constexpr int kReduceBlock = 256;
int64_t partial_count(int64_t n_items, int block);

// Red-black sweeps in place on phi.  With a scratch array `tmp` of the same
// size and n >= 16, each sweep is one fused LDS-tiled kernel reading one
// buffer and writing the other; otherwise two half-sweep kernels.
bool tiled_smoother(int n);
// A zero-guess V-cycle over n0, n0/2, ..., 4 (n0 = 8 or 16) inside one
// workgroup, reading the rhs b and writing the correction e (oct-major);
// G4: pseudo-inverse of the 4^3 operator at spacing h0 * n0 / 4.
bool small_vcycle(int n);
template <typename T>
void u_vcycle_small(int n0, double h0, const T* b, T* e, const T* G4, int nu_pre, int nu_post, hipStream_t s);
// one fused tiled sweep src -> dst (n >= 16); src == nullptr: the incoming phi
// is zero (not read); with `partials` (one f64 per block,
// tiled_sweep_blocks(n) of them) it also sums ||b - L src||^2; with
// `ec_prolong` (coarse grid n/2) the sweep applies to src + P ec_prolong
int64_t tiled_sweep_blocks(int n);
// add64: the swept values are added to this f64 array instead of being
// written to dst (the last sweep of an FP32 correction cycle)
// Returns the number of partial sums written (= blocks launched); at most
// partial_count(n^3, kReduceBlock).
template <typename T>
int64_t u_sweep_tiled(int n, double h, const T* src, const T* b, T* dst, double* partials, hipStream_t s,
                      const T* ec_prolong = nullptr, double* add64 = nullptr);
// `sweeps` tiled sweeps starting from *cur (zero_first: the incoming phi is
// zero and *cur is not read; ec: prolongation applied to the incoming phi),
// ping-ponging between *cur and *other; on return *cur points at the buffer
// that holds the result.  add_last (sweeps >= 1): the last sweep adds its
// result to this f64 array instead (*cur then holds the previous iterate).
template <typename T>
void u_sweeps_tiled(int n, double h, T** cur, T** other, const T* b, int sweeps, bool zero_first, const T* ec,
                    hipStream_t s, double* add_last = nullptr);
template <typename T>
void u_smooth(int n, double h, T* phi, const T* b, int sweeps, hipStream_t s, T* tmp);
template <typename T>
void u_smooth_zero_guess(int n, double h, T* phi, const T* b, int sweeps, hipStream_t s, T* tmp);
template <typename T>
int64_t u_resid_restrict(int n, double h, const T* phi, const T* b, T* bc, double* partials,
                         hipStream_t s);   // returns the number of partial sums written
template <typename T>
void u_prolong(int n, const T* ec, T* e, hipStream_t s);
template <typename T>
void u_coarse_solve(int n, const T* G, const T* b, T* e, hipStream_t s);
template <typename T>
void fill_zero(T* p, int64_t n, hipStream_t s);

// f = c (rho - mean) with mean read from d_mean (device); partial sums of f^2
// (f may be NULL: the sums only); returns how many partials it wrote (at most
// partial_count(n_cells, kReduceBlock))
int64_t u_rhs(int64_t n_cells, const double* rho, const double* d_mean, double c, double* f,
              double* partials, hipStream_t s);
// partial sums of x (f64 input, n >= 1); returns how many partials it wrote
// (at most partial_count(n, kReduceBlock))
int64_t partial_sum(int64_t n, const double* x, double* partials, hipStream_t s);
// out[slot] = scale * sum(partials[0..count))
void reduce_final(const double* partials, int64_t count, double scale, double* out, int slot,
                  hipStream_t s);
// x -= d_mean[0]
void sub_mean(int64_t n, double* x, const double* d_mean, hipStream_t s);
// phi64 += e32
void add_correction(int64_t n, double* phi, const float* e, hipStream_t s);
// ||f - L phi||^2 and ||f||^2 per tile (partials, partials_f) with f = c (rho -
// *d_mean) formed on the fly (n >= 16); returns the number of tiles
int64_t u_resid_from_rho(int n, double h, const double* phi, const double* rho, double c, const double* d_mean,
                         double* partials, double* partials_f, hipStream_t s);
// Grids (n >= 512) whose mixed-precision outer residual runs fused with the
// first FP32 sweep of the correction cycle (zero guess): r32 = RNE(f - L phi)
// and e32 = that sweep's result (the cycle's level-0 iterate after one
// pre-smoothing sweep), partial sums of r^2; returns the number of partials.
bool fused_outer_resid(int n);
int64_t u_outer_resid_sweep(int n, double h, const double* phi, const double* f, float* r32, float* e32,
                            double* partials, hipStream_t s);
// r32 = f - L phi (f64 arithmetic), partial sums of r^2 (periodic grid)
int64_t u_outer_resid(int n, double h, const double* phi, const double* f, float* r32,
                      double* partials, hipStream_t s);   // returns the number of partial sums written

// dense (x n + y) n + z <-> oct-major copy of an n^3 f64 field (n a power of two >= 2)
void u_layout(int n, bool to_oct, const double* in, double* out, hipStream_t s);

// pseudo-inverse of the periodic 7-point operator on n^3 cells (oct-major order)
std::vector<double> coarse_pinv(int n, double h);

// ---------------------------------------------------------------------------
// oct-list levels (amr.hip)
// ---------------------------------------------------------------------------
void morton_keys(int64_t n, const int32_t* ijk, uint64_t* keys, hipStream_t s);
void oct_validate(int64_t n, const int32_t* ijk, int n_dim, int* flag, hipStream_t s);
size_t hash_slot_bytes();
void hash_build(int64_t n, const uint64_t* keys, void* table, int64_t cap, int* flag, hipStream_t s);
void hash_lookup_many(int64_t n, const uint64_t* q, const void* table, int64_t cap, int32_t* out, hipStream_t s);
void nbr_from_hash(int64_t n, const uint64_t* keys, int n_dim, const void* table, int64_t cap, int32_t* nbr,
                   int32_t* missing, hipStream_t s);
void exclusive_scan_i32(int64_t n, const int32_t* in, int32_t* out, hipStream_t s);
// pcells: the parent's cells per dimension in its key frame; shift: this
// level's frame origin (octs) minus twice the parent's (parent cells)
void ghost_stencils(int64_t n, const uint64_t* keys, int n_dim, const int32_t* first, int32_t* nbr,
                    bool parent_uniform, const void* ptable, int64_t pcap, int pcells, const int (&shift)[3],
                    int32_t* gidx, int* flag, hipStream_t s);
void ghost_values(int64_t n_ghost, const int32_t* gidx, const double* phi_parent, double* gval, hipStream_t s);
// per-workgroup ||f - (ghost neighbour sum) / h^2||^2 of a finest refined level
// (ghost faces encoded in nbr, values in ghost); returns the number of partials
int64_t oct_rhs_norm2(int64_t n, double h, const double* f, const int32_t* nbr, const double* ghost, double* partials,
                      hipStream_t s);
int64_t unique_parent_keys(int64_t n, const uint64_t* keys, DevBuf& out, int key_bits, bool sorted,
                           bool out_scratch, hipStream_t s, int drop = 3);
void fathers(int64_t n, const uint64_t* keys, const uint64_t* ckeys, int64_t nc, int32_t* father, int* flag,
             hipStream_t s);
// coarse level-set mask: -1 everywhere, father cells = mean of the children's masks (fine_lsm NULL = all +1)
void coarse_level_set(int64_t n_fine, const int32_t* father, const float* fine_lsm, int64_t n_coarse,
                      float* coarse_lsm, hipStream_t s);
// active bits (mask > 0) and the per-cell diagonal of the coarse error operator
template <typename T>
void level_set_operator(int64_t n, const int32_t* nbr, const float* lsm, uint8_t* mask, T* diag, hipStream_t s);
void nbr_sorted(int64_t n, const uint64_t* keys, int n_dim, int32_t* nbr, int32_t* nbr27, hipStream_t s);
// *count += active cells (set mask bits) of n octs
void count_active(int64_t n, const uint8_t* mask, unsigned long long* count, hipStream_t s);
int coarsest_oct_capacity();
// Bricks of 4 x 4 x 4 octs on a lattice shifted by `shift` (bit a: one oct
// along axis a): sorted unique keys of (oct + shift) >> 2 (returns the count;
// synchronises), and each brick's 6 x 6 x 6 oct box map (oct index or -1),
// looked up in the level's hash table (table != NULL) or in its sorted keys.
// n_dim >= 4 (a brick then holds distinct octs).
int64_t brick_keys(int64_t n, const uint64_t* keys, bool sorted, int n_dim, int shift, DevBuf& out,
                   hipStream_t s);
void brick_map(int64_t n_bricks, const uint64_t* bkeys, int n_dim, int shift, const void* table, int64_t cap,
               const uint64_t* sorted_keys, int64_t n_sorted, int32_t* map, hipStream_t s);
// The shift in [0, 8) whose lattice covers the level's octs with the fewest
// bricks (ties: the smallest; 0 on levels under 4096 octs or wider than 1024
// octs per dimension).  Synchronises.
int choose_brick_shift(int64_t n, const uint64_t* keys, int n_dim, hipStream_t s);
// Per-brick ghost lists (finest refined level): first[b * 216] .. first[(b + 1)
// * 216] index entries (box cell, ghost value index).  Returns the entry count.
int64_t brick_ghosts(int64_t n_bricks, const int32_t* map, const int32_t* nbr, DevBuf& first, DevBuf& cell,
                     DevBuf& gv, hipStream_t s);
struct BrickGhosts {
  const int32_t* first = nullptr;   // [n_bricks * 216 + 1] list offsets
  const int32_t* cell = nullptr;    // box cell of each entry
  const double* val = nullptr;      // value of each entry (gathered per solve); NULL: absent neighbours count 0
};
// out[e] = gval[gidx[e]] for the n entries of the brick ghost lists
void brick_ghost_pack(int64_t n, const int32_t* gidx, const double* gval, double* out, hipStream_t s);
// One red-black sweep of every brick: src -> dst (src == NULL: zero guess).
// mask/diag NULL: all cells active, diagonal 6.  With `partials`, also
// ||b - L src||^2 per brick (partials[brick]) of the incoming src.  With `ec`
// (and the coarse map `cmap` of brick_cmap, built with the level's brick
// shift `cshift`), the sweep applies to src plus the trilinear prolongation
// of the coarse correction ec.  With `add64`, the swept values are added to
// that f64 array (same layout) instead of being written to dst.
template <typename T>
void brick_sweep(int64_t n_bricks, const int32_t* map, double h, const T* src, const T* b, T* dst,
                 const uint8_t* mask, const T* diag, const BrickGhosts& gh, hipStream_t s,
                 double* partials = nullptr, const int32_t* cmap = nullptr, int cshift = 0, const T* ec = nullptr,
                 double* add64 = nullptr);
// cmap[b][125]: the coarse octs (sorted keys ckeys of the next level, n_dim_c
// octs per dimension) of brick b's 5 x 5 x 5-oct coarse box, -1 where absent
// or outside the 8^3-cell window that a prolongation into the box reads
void brick_cmap(int64_t n_bricks, const uint64_t* bkeys, int n_dim_c, int shift, const uint64_t* ckeys,
                int64_t n_coarse, int32_t* cmap, hipStream_t s);
// The small levels at the bottom of a refined level's hierarchy, cycled in
// one workgroup with every value in LDS ("tail").  Compact cell indices run
// over all tail levels (level k holds [off[k], off[k + 1]), its red cells
// first).  One table blob, copied as is into LDS: the diagonal dg [n] (cycle
// precision), nb [n][6] same-level neighbours (-x, +x, -y, +y, -z, +z; -1
// absent or inactive), kids [n - off[1]][8] (cells of levels >= 1) the 8
// cells of the finer level whose residuals restrict into the cell, par
// [off[last]][8] (cells of levels < last) the coarse cells of the trilinear
// prolongation in the order (0,0,0), (0,0,z), (0,y,0), (0,y,z), (x,0,0),
// (x,0,z), (x,y,0), (x,y,z), each offset towards the fine cell's side; all
// indices int16.  The first level's right-hand side arrives compact (bt,
// written by the level above's restriction through its compact father map);
// cell0[i] is the flat cell of tail cell i in the first level's e array.
constexpr int kTailMaxLevels = 8;
struct TailArgs {
  int levels = 0;
  int nu_pre = 0, nu_post = 0, last_sweeps = 0;
  int ns = 0;       // stride of e and b in LDS: n rounded up to 4
  int blob16 = 0;   // 16-byte units of the table blob
  int off[kTailMaxLevels + 1] = {};
  int nred[kTailMaxLevels] = {};
  double h2[kTailMaxLevels] = {};
  double inv_h2[kTailMaxLevels] = {};
};
// bytes of the table blob, and of the LDS, of a tail of n cells, n_first on
// its first level and n_last on its last, for elements of elem_bytes; and
// the most LDS a tail may take
size_t tail_blob_bytes(int64_t n, int64_t n_first, int64_t n_last, size_t elem_bytes);
size_t tail_lds_bytes(int64_t n, int64_t n_first, int64_t n_last, size_t elem_bytes);
size_t tail_lds_limit();
// One V-cycle over the tail levels from bt; e of the first level scattered
// into e0 (its active cells only).
template <typename T>
void oct_tail(const TailArgs& a, const void* blob, const T* bt, const int32_t* cell0, T* e0, hipStream_t s);
// Residual of e per brick: restricted into bc[father] (if bc), per cell in
// FP32 (if r32), ||r||^2 per brick into partials[brick] (if partials).
template <typename T>
void brick_resid(int64_t n_bricks, const int32_t* map, double h, const T* e, const T* b, const uint8_t* mask,
                 const T* diag, const BrickGhosts& gh, const int32_t* father, T* bc, float* r32, double* partials,
                 hipStream_t s);
// Direct FFT solve of a periodic level (n^3 cells, oct-major f and phi, n a
// power of two in [8, fft_max_n()]): phi = exact solution of L_h phi = f with
// mean 0.  work: fft_work_bytes(n) (n^2 rows of the n/2 + 1 frequencies of a
// real row, padded); tw, lam from fft_tables.
int fft_max_n();
size_t fft_work_bytes(int n);
void fft_tables(int n, double h, DevBuf& tw, DevBuf& lam, hipStream_t s);
// src: f, or rho with gscale = four_pi_G (the mean only moves the zero mode,
// which the solve sets to 0); gscale multiplies the result.  With `partials`,
// the sum of src over each x-pass workgroup ((n/2)^2 of them) for the mean.
void fft_solve(int n, const double* src, double gscale, double* phi, void* work, const void* tw, const double* lam,
               double* partials, hipStream_t s);
// g = -grad(phi) by central differences, component-major [3][cells]:
// periodic n^3 level (octs lexicographic) / an oct level with its neighbour
// cache and ghost values (ghost faces encoded as nbr <= -2)
void u_force(int n, double h, const double* phi, double* g, hipStream_t s);
void oct_force(int64_t n, double h, const double* phi, const int32_t* nbr, const double* ghost, double* g,
               hipStream_t s);
// copy a neighbour cache with ghost encodings replaced by -1
void nbr_export(int64_t n, const int32_t* nbr, int32_t* out, hipStream_t s);

template <typename T>
void oct_smooth(int64_t n, double h, T* e, const T* b, const int32_t* nbr, const uint8_t* mask,
                const T* diag, const double* ghost, int sweeps, hipStream_t s);
template <typename T>
void oct_resid(int64_t n, double h, const T* e, const T* b, const int32_t* nbr, const uint8_t* mask,
               const T* diag, const double* ghost, const int32_t* father, T* bc, float* r32,
               double* partials, hipStream_t s);
template <typename T>
void oct_prolong(int64_t n, const int32_t* father, const int32_t* cnbr27, const T* ec, T* e, const uint8_t* mask,
                 hipStream_t s);
template <typename T>
void oct_coarsest(int64_t n, double h, T* e, const T* b, const int32_t* nbr, const uint8_t* mask,
                  const T* diag, int sweeps, hipStream_t s);

}  // namespace mg

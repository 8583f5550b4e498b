// A Morton-key -> grid-index table maintained incrementally (appendix
// "Per-level hash table and replacement functions": insert when a grid is
// made, delete when it is killed, a rebuild that drops deleted entries), with
// 64-bit keys (B = 21 bits per coordinate) or 128-bit keys (B = 42, section
// "Morton key encoding and neighbour arithmetic"; two words, low first).
//
// * Open addressing with linear probing; capacity a power of two; the slot is
//   hash_func(k) & (capacity - 1) with k the key itself (64-bit) or the XOR of
//   its two words (128-bit).
// * A slot's state lives in its high key word: all ones = empty, all ones
//   minus one = deleted.  Valid keys leave bit 63 (64-bit keys) or bits 62-63
//   of the high word (128-bit keys, 126 key bits) clear, so neither value is a
//   key.
// * Insert is three launches, so that no thread compares a key another
//   thread is still writing: (1) keys already present take the new value and
//   the others are counted (the host grows the table for them if needed);
//   (2) every other key claims the first empty slot on its probe sequence by
//   a 64-bit compare-and-swap of the high word, then writes its low word and
//   value; (3) a key repeated in the batch has claimed several slots on the
//   same probe sequence: every claimant but the first in probe order turns
//   its slot into a deleted one.  Deleted slots are not reused; the table is
//   rebuilt (doubling as needed) when live plus deleted slots would pass the
//   fill limit.
// * Neighbour lookup (equation nbor_precompute's keys): decode, step one
//   coordinate with periodic wrap at the level's extent, re-encode, look up.
#include <algorithm>
#include <memory>
#include <vector>

#include "mg_internal.h"

namespace mg {

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kEmpty = ~0ull;
constexpr uint64_t kDeleted = ~0ull - 1;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <int W>
struct HSlot;
template <>
struct HSlot<1> {
  unsigned long long hi;   // the key
  int32_t val;
  int32_t pad;
};
template <>
struct HSlot<2> {
  unsigned long long hi;   // key bits 64..127
  unsigned long long lo;   // key bits 0..63
  int32_t val;
  int32_t pad;
};

// counters: slots claimed, claims undone as repeats, keys erased, bad keys,
// keys left to claim after the update pass
enum { kClaimed = 0, kRepeats = 1, kErased = 2, kBadKeys = 3, kPending = 4, kNumCounters = 5 };

// Each counter has kCopies copies, one per 128-byte line; the host sums them.
// Atomics on one address serialise in L2 (several ns each), so a wave adds
// its count once, to the copy picked by its index.
constexpr int kCopies = 64, kCopyStride = 16;   // u64 words between copies
__device__ __forceinline__ void wave_count(unsigned long long* cnt, int k, bool pred) {
  const unsigned long long act = __ballot(1);
  const unsigned long long m = __ballot(pred);
  if (m != 0 && (int)__lane_id() == __ffsll((long long)act) - 1) {
    const unsigned copy = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & (kCopies - 1);
    atomicAdd(&cnt[(k * kCopies + copy) * kCopyStride], (unsigned long long)__popcll(m));
  }
}

template <int W>
__device__ __forceinline__ void read_key(const uint64_t* __restrict__ keys, int64_t i, uint64_t& hi, uint64_t& lo) {
  if constexpr (W == 1) {
    hi = keys[i];
    lo = 0;
  } else {
    lo = keys[2 * i];
    hi = keys[2 * i + 1];
  }
}

template <int W>
__device__ __forceinline__ bool valid_key(uint64_t hi) {
  return W == 1 ? (hi >> 63) == 0 : (hi >> 62) == 0;
}

template <int W>
__device__ __forceinline__ uint64_t home(uint64_t hi, uint64_t lo, uint64_t mask) {
  return hash64(W == 1 ? hi : (hi ^ lo)) & mask;
}

// first slot on the probe sequence holding the key, or -1 (an empty slot ends it)
template <int W>
__device__ __forceinline__ int64_t find_slot(const HSlot<W>* __restrict__ t, uint64_t mask, uint64_t hi,
                                             uint64_t lo) {
  uint64_t s = home<W>(hi, lo, mask);
  for (uint64_t p = 0; p <= mask; ++p) {
    const uint64_t h = t[s].hi;
    if (h == kEmpty) return -1;
    if (h == hi) {
      if constexpr (W == 1) return (int64_t)s;
      else if (t[s].lo == lo) return (int64_t)s;
    }
    s = (s + 1) & mask;
  }
  return -1;
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_clear(int64_t cap, HSlot<W>* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  t[i].hi = kEmpty;
  if constexpr (W == 2) t[i].lo = 0;
  t[i].val = -1;
  t[i].pad = 0;
}

// (1) update keys already present; mark the others (claim[i] = -2) for step 2
template <int W>
__global__ __launch_bounds__(kBlock) void k_update(int64_t n, const uint64_t* __restrict__ keys,
                                                   const int32_t* __restrict__ vals, HSlot<W>* __restrict__ t,
                                                   uint64_t mask, int64_t* __restrict__ claim,
                                                   unsigned long long* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t hi, lo;
  read_key<W>(keys, i, hi, lo);
  const bool valid = valid_key<W>(hi);
  bool pending = false;
  if (valid) {
    const int64_t s = find_slot<W>(t, mask, hi, lo);
    if (s >= 0) t[s].val = vals[i];
    pending = s < 0;
  }
  claim[i] = pending ? -2 : -1;
  wave_count(cnt, kBadKeys, !valid);
  wave_count(cnt, kPending, pending);
}

// (2) claim the first empty slot on the probe sequence (the host keeps the
// fill below 1, so one exists)
template <int W>
__global__ __launch_bounds__(kBlock) void k_claim(int64_t n, const uint64_t* __restrict__ keys,
                                                  const int32_t* __restrict__ vals, HSlot<W>* __restrict__ t,
                                                  uint64_t mask, int64_t* __restrict__ claim,
                                                  unsigned long long* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool claimed = false;
  if (claim[i] == -2) {
    uint64_t hi, lo;
    read_key<W>(keys, i, hi, lo);
    uint64_t s = home<W>(hi, lo, mask);
    int64_t got = -1;   // stays -1 only if the table were full, which the host prevents
    for (uint64_t p = 0; p <= mask; ++p) {
      if (t[s].hi == kEmpty && atomicCAS(&t[s].hi, kEmpty, (unsigned long long)hi) == kEmpty) {
        if constexpr (W == 2) t[s].lo = lo;
        t[s].val = vals[i];
        got = (int64_t)s;
        break;
      }
      s = (s + 1) & mask;
    }
    claim[i] = got;
    claimed = got >= 0;
  }
  wave_count(cnt, kClaimed, claimed);
}

// (3) a repeated key keeps only its first slot in probe order
template <int W>
__global__ __launch_bounds__(kBlock) void k_dedupe(int64_t n, const uint64_t* __restrict__ keys,
                                                   HSlot<W>* __restrict__ t, uint64_t mask,
                                                   const int64_t* __restrict__ claim,
                                                   unsigned long long* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t mine = claim[i];
  bool undone = false;
  if (mine >= 0) {
    uint64_t hi, lo;
    read_key<W>(keys, i, hi, lo);
    if (find_slot<W>(t, mask, hi, lo) != mine) {
      t[mine].hi = kDeleted;
      undone = true;
    }
  }
  wave_count(cnt, kRepeats, undone);
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_erase(int64_t n, const uint64_t* __restrict__ keys,
                                                  HSlot<W>* __restrict__ t, uint64_t mask,
                                                  unsigned long long* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t hi, lo;
  read_key<W>(keys, i, hi, lo);
  const bool valid = valid_key<W>(hi);
  bool erased = false;
  if (valid) {
    const int64_t s = find_slot<W>(t, mask, hi, lo);
    // a key repeated in the batch finds the same slot: one compare-and-swap wins
    if (s >= 0) erased = atomicCAS(&t[s].hi, (unsigned long long)hi, (unsigned long long)kDeleted) == hi;
  }
  wave_count(cnt, kBadKeys, !valid);
  wave_count(cnt, kErased, erased);
}

template <int W>
__global__ __launch_bounds__(kBlock) void k_lookup(int64_t n, const uint64_t* __restrict__ keys,
                                                   const HSlot<W>* __restrict__ t, uint64_t mask,
                                                   int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t hi, lo;
  read_key<W>(keys, i, hi, lo);
  const int64_t s = valid_key<W>(hi) ? find_slot<W>(t, mask, hi, lo) : -1;
  out[i] = s >= 0 ? t[s].val : -1;
}

// move the live slots of a table into an empty one (keys are distinct)
template <int W>
__global__ __launch_bounds__(kBlock) void k_reinsert(int64_t old_cap, const HSlot<W>* __restrict__ from,
                                                     HSlot<W>* __restrict__ to, uint64_t mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= old_cap) return;
  const uint64_t hi = from[i].hi;
  if (hi == kEmpty || hi == kDeleted) return;
  uint64_t lo = 0;
  if constexpr (W == 2) lo = from[i].lo;
  uint64_t s = home<W>(hi, lo, mask);
  for (uint64_t p = 0; p <= mask; ++p) {
    if (atomicCAS(&to[s].hi, kEmpty, (unsigned long long)hi) == kEmpty) {
      if constexpr (W == 2) to[s].lo = lo;
      to[s].val = from[i].val;
      return;
    }
    s = (s + 1) & mask;
  }
}

// ---- 128-bit keys: x bits 0..20 -> key bits 3b, bit 21 -> bit 63, bits
// 22..41 -> high-word bits 3(b-22)+2; y, z bits 0..20 -> 3b+1, 3b+2 and bits
// 21..41 -> high-word bits 3(b-21), 3(b-21)+1
__device__ __forceinline__ void morton128(uint64_t x, uint64_t y, uint64_t z, uint64_t& hi, uint64_t& lo) {
  lo = spread3(x & 0x1fffff) | (spread3(y & 0x1fffff) << 1) | (spread3(z & 0x1fffff) << 2) | (((x >> 21) & 1) << 63);
  hi = (spread3((x >> 22) & 0xfffff) << 2) | spread3((y >> 21) & 0x1fffff) | (spread3((z >> 21) & 0x1fffff) << 1);
}
__device__ __forceinline__ void unmorton128(uint64_t hi, uint64_t lo, uint64_t& x, uint64_t& y, uint64_t& z) {
  x = (uint64_t)compact3(lo) | (((lo >> 63) & 1) << 21) | ((uint64_t)compact3(hi >> 2) << 22);
  y = (uint64_t)compact3(lo >> 1) | ((uint64_t)compact3(hi) << 21);
  z = (uint64_t)compact3(lo >> 2) | ((uint64_t)compact3(hi >> 1) << 21);
}

__global__ __launch_bounds__(kBlock) void k_morton128(int64_t n, const int64_t* __restrict__ ijk,
                                                      uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t hi, lo;
  morton128((uint64_t)ijk[3 * i], (uint64_t)ijk[3 * i + 1], (uint64_t)ijk[3 * i + 2], hi, lo);
  keys[2 * i] = lo;
  keys[2 * i + 1] = hi;
}

// neighbour grid indices in directions -x, +x, -y, +y, -z, +z (-1: absent);
// dmask = octs per dimension - 1 (a power of two minus one)
template <int W>
__global__ __launch_bounds__(kBlock) void k_neighbours(int64_t n, const uint64_t* __restrict__ keys,
                                                       uint64_t dmask, const HSlot<W>* __restrict__ t,
                                                       uint64_t mask, int32_t* __restrict__ nbr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t hi, lo;
  read_key<W>(keys, i, hi, lo);
  if (!valid_key<W>(hi)) {
    for (int j = 0; j < 6; ++j) nbr[i * 6 + j] = -1;
    return;
  }
  uint64_t c[3];
  if constexpr (W == 1) {
    int x, y, z;
    unmorton(hi, x, y, z);
    c[0] = (uint64_t)x;
    c[1] = (uint64_t)y;
    c[2] = (uint64_t)z;
  } else {
    unmorton128(hi, lo, c[0], c[1], c[2]);
  }
  for (int j = 0; j < 6; ++j) {
    uint64_t q[3] = {c[0], c[1], c[2]};
    const int d = j >> 1;
    q[d] = (q[d] + ((j & 1) ? 1ull : dmask)) & dmask;   // +-1 with periodic wrap
    uint64_t khi, klo;
    if constexpr (W == 1) {
      khi = morton((uint32_t)q[0], (uint32_t)q[1], (uint32_t)q[2]);
      klo = 0;
    } else {
      morton128(q[0], q[1], q[2], khi, klo);
    }
    const int64_t s = find_slot<W>(t, mask, khi, klo);
    nbr[i * 6 + j] = s >= 0 ? t[s].val : -1;
  }
}

}  // namespace
}  // namespace mg

using namespace mg;

struct mg_hash_s {
  int W = 1;
  double max_load = 0.7;
  hipStream_t stream = nullptr;
  DevBuf slots;
  int64_t cap = 0, n_live = 0, n_deleted = 0;
  DevBuf claim;              // i64 per key of the largest insert so far
  DevBuf cnt;                // u64 [kNumCounters]
  size_t slot_bytes() const { return W == 1 ? sizeof(HSlot<1>) : sizeof(HSlot<2>); }
  uint64_t mask() const { return (uint64_t)cap - 1; }

  void clear_table(DevBuf& buf, int64_t c) {
    buf.alloc((size_t)c * slot_bytes());
    if (W == 1) hipLaunchKernelGGL(k_clear<1>, dim3(grid_for(c)), dim3(kBlock), 0, stream, c, buf.as<HSlot<1>>());
    else hipLaunchKernelGGL(k_clear<2>, dim3(grid_for(c)), dim3(kBlock), 0, stream, c, buf.as<HSlot<2>>());
    check_launch();
  }
  // rebuild at capacity new_cap from the live slots (drops deleted ones)
  void rehash(int64_t new_cap) {
    DevBuf fresh;
    clear_table(fresh, new_cap);
    const uint64_t m = (uint64_t)new_cap - 1;
    if (cap > 0) {
      if (W == 1)
        hipLaunchKernelGGL(k_reinsert<1>, dim3(grid_for(cap)), dim3(kBlock), 0, stream, cap, slots.as<HSlot<1>>(),
                           fresh.as<HSlot<1>>(), m);
      else
        hipLaunchKernelGGL(k_reinsert<2>, dim3(grid_for(cap)), dim3(kBlock), 0, stream, cap, slots.as<HSlot<2>>(),
                           fresh.as<HSlot<2>>(), m);
      check_launch();
      MG_HIP(hipStreamSynchronize(stream));   // the old table is read until here
    }
    slots = std::move(fresh);
    cap = new_cap;
    n_deleted = 0;
  }
  // capacity for `live` entries under the fill limit, at least `floor`
  int64_t capacity_for(int64_t live, int64_t floor) const {
    int64_t c = std::max<int64_t>(floor, 16);
    while ((double)live > max_load * (double)c) c *= 2;
    return c;
  }
  static constexpr size_t kCounterWords = (size_t)kNumCounters * kCopies * kCopyStride;
  void read_counters(unsigned long long (&h)[kNumCounters]) {
    std::vector<unsigned long long> all(kCounterWords);
    MG_HIP(hipMemcpyAsync(all.data(), cnt.p, kCounterWords * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          stream));
    MG_HIP(hipStreamSynchronize(stream));
    for (int k = 0; k < kNumCounters; ++k) {
      h[k] = 0;
      for (int c = 0; c < kCopies; ++c) h[k] += all[((size_t)k * kCopies + c) * kCopyStride];
    }
  }
  void zero_counters() {
    MG_HIP(hipMemsetAsync(cnt.p, 0, kCounterWords * sizeof(unsigned long long), stream));
  }
};

namespace {
bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }
}  // namespace

// Hash of each key (equation hash_func after the reduction to 64 bits), the
// value whose low bits pick a key's home slot in both tables.
template <int W>
__global__ __launch_bounds__(kBlock) void k_hash_values(int64_t n, const uint64_t* __restrict__ keys,
                                                        uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t hi, lo;
  read_key<W>(keys, i, hi, lo);
  out[i] = hash64(W == 1 ? hi : (hi ^ lo));
}

extern "C" {

mg_status_t mg_hash_create(int32_t key_words, int64_t capacity, double max_load, void* stream, mg_hash_t* out) {
  MG_API_BEGIN
  MG_REQUIRE(out != nullptr, "mg_hash_create: out is NULL");
  *out = nullptr;
  MG_REQUIRE(key_words == 1 || key_words == 2, "mg_hash_create: key_words must be 1 (64-bit) or 2 (128-bit)");
  MG_REQUIRE(max_load > 0.0 && max_load <= 0.9, "mg_hash_create: max_load must be in (0, 0.9]");
  MG_REQUIRE(capacity >= 0 && capacity <= ((int64_t)1 << 40), "mg_hash_create: capacity out of range");
  std::unique_ptr<mg_hash_s> H(new mg_hash_s());
  H->W = key_words;
  H->max_load = max_load;
  H->stream = (hipStream_t)stream;
  int64_t c = 16;
  while (c < capacity) c *= 2;
  H->cnt.alloc(mg_hash_s::kCounterWords * sizeof(unsigned long long));
  H->rehash(c);
  MG_HIP(hipStreamSynchronize(H->stream));
  *out = H.release();
  return MG_OK;
  MG_API_END
}

void mg_hash_destroy(mg_hash_t H) {
  if (H && H->stream) (void)hipStreamSynchronize(H->stream);
  delete H;
}

mg_status_t mg_hash_insert(mg_hash_t H, int64_t n, const uint64_t* d_keys, const int32_t* d_vals) {
  MG_API_BEGIN
  MG_REQUIRE(H != nullptr, "mg_hash_insert: handle is NULL");
  MG_REQUIRE(n >= 0, "mg_hash_insert: n must be >= 0");
  if (n == 0) return MG_OK;
  MG_REQUIRE(d_keys && d_vals && aligned8(d_keys), "mg_hash_insert: NULL or misaligned argument");
  if (H->claim.bytes < (size_t)n * sizeof(int64_t)) H->claim.alloc((size_t)n * sizeof(int64_t));
  H->zero_counters();
  unsigned long long* cnt = H->cnt.as<unsigned long long>();
  int64_t* claim = H->claim.as<int64_t>();
  const dim3 g(grid_for(n)), b(kBlock);
  // (1) present keys take their values; the rest are counted
  if (H->W == 1)
    hipLaunchKernelGGL(k_update<1>, g, b, 0, H->stream, n, d_keys, d_vals, H->slots.as<HSlot<1>>(), H->mask(),
                       claim, cnt);
  else
    hipLaunchKernelGGL(k_update<2>, g, b, 0, H->stream, n, d_keys, d_vals, H->slots.as<HSlot<2>>(), H->mask(),
                       claim, cnt);
  check_launch();
  unsigned long long h[kNumCounters];
  H->read_counters(h);
  // room for every key left to claim (repeats included) within the fill limit
  const int64_t pending = (int64_t)h[kPending];
  if ((double)(H->n_live + H->n_deleted + pending) > H->max_load * (double)H->cap)
    H->rehash(H->capacity_for(H->n_live + pending, H->cap));
  // (2) claims, (3) repeats undone
  const uint64_t m = H->mask();
  if (pending > 0) {
    if (H->W == 1) {
      HSlot<1>* t = H->slots.as<HSlot<1>>();
      hipLaunchKernelGGL(k_claim<1>, g, b, 0, H->stream, n, d_keys, d_vals, t, m, claim, cnt);
      hipLaunchKernelGGL(k_dedupe<1>, g, b, 0, H->stream, n, d_keys, t, m, claim, cnt);
    } else {
      HSlot<2>* t = H->slots.as<HSlot<2>>();
      hipLaunchKernelGGL(k_claim<2>, g, b, 0, H->stream, n, d_keys, d_vals, t, m, claim, cnt);
      hipLaunchKernelGGL(k_dedupe<2>, g, b, 0, H->stream, n, d_keys, t, m, claim, cnt);
    }
    check_launch();
    H->read_counters(h);
  }
  H->n_live += (int64_t)h[kClaimed] - (int64_t)h[kRepeats];
  H->n_deleted += (int64_t)h[kRepeats];
  MG_REQUIRE(h[kBadKeys] == 0, "mg_hash_insert: a key has its sentinel bits set (not a Morton key); it was skipped");
  return MG_OK;
  MG_API_END
}

mg_status_t mg_hash_erase(mg_hash_t H, int64_t n, const uint64_t* d_keys) {
  MG_API_BEGIN
  MG_REQUIRE(H != nullptr, "mg_hash_erase: handle is NULL");
  MG_REQUIRE(n >= 0, "mg_hash_erase: n must be >= 0");
  if (n == 0) return MG_OK;
  MG_REQUIRE(d_keys && aligned8(d_keys), "mg_hash_erase: NULL or misaligned argument");
  H->zero_counters();
  unsigned long long* cnt = H->cnt.as<unsigned long long>();
  if (H->W == 1)
    hipLaunchKernelGGL(k_erase<1>, dim3(grid_for(n)), dim3(kBlock), 0, H->stream, n, d_keys,
                       H->slots.as<HSlot<1>>(), H->mask(), cnt);
  else
    hipLaunchKernelGGL(k_erase<2>, dim3(grid_for(n)), dim3(kBlock), 0, H->stream, n, d_keys,
                       H->slots.as<HSlot<2>>(), H->mask(), cnt);
  check_launch();
  unsigned long long h[kNumCounters];
  H->read_counters(h);
  H->n_live -= (int64_t)h[kErased];
  H->n_deleted += (int64_t)h[kErased];
  MG_REQUIRE(h[kBadKeys] == 0, "mg_hash_erase: a key has its sentinel bits set (not a Morton key); it was skipped");
  return MG_OK;
  MG_API_END
}

mg_status_t mg_hash_lookup(mg_hash_t H, int64_t n, const uint64_t* d_keys, int32_t* d_vals) {
  MG_API_BEGIN
  MG_REQUIRE(H != nullptr, "mg_hash_lookup: handle is NULL");
  MG_REQUIRE(n >= 0, "mg_hash_lookup: n must be >= 0");
  if (n == 0) return MG_OK;
  MG_REQUIRE(d_keys && d_vals && aligned8(d_keys), "mg_hash_lookup: NULL or misaligned argument");
  if (H->W == 1)
    hipLaunchKernelGGL(k_lookup<1>, dim3(grid_for(n)), dim3(kBlock), 0, H->stream, n, d_keys,
                       H->slots.as<HSlot<1>>(), H->mask(), d_vals);
  else
    hipLaunchKernelGGL(k_lookup<2>, dim3(grid_for(n)), dim3(kBlock), 0, H->stream, n, d_keys,
                       H->slots.as<HSlot<2>>(), H->mask(), d_vals);
  check_launch();
  return MG_OK;
  MG_API_END
}

mg_status_t mg_hash_neighbours(mg_hash_t H, int64_t n, const uint64_t* d_keys, int64_t n_dim, int32_t* d_nbr) {
  MG_API_BEGIN
  MG_REQUIRE(H != nullptr, "mg_hash_neighbours: handle is NULL");
  MG_REQUIRE(n >= 0, "mg_hash_neighbours: n must be >= 0");
  MG_REQUIRE(is_pow2(n_dim) && n_dim <= ((int64_t)1 << (H->W == 1 ? 21 : 42)),
             "mg_hash_neighbours: n_dim must be a power of two within the key's coordinate range");
  if (n == 0) return MG_OK;
  MG_REQUIRE(d_keys && d_nbr && aligned8(d_keys), "mg_hash_neighbours: NULL or misaligned argument");
  const uint64_t dm = (uint64_t)n_dim - 1;
  if (H->W == 1)
    hipLaunchKernelGGL(k_neighbours<1>, dim3(grid_for(n)), dim3(kBlock), 0, H->stream, n, d_keys, dm,
                       H->slots.as<HSlot<1>>(), H->mask(), d_nbr);
  else
    hipLaunchKernelGGL(k_neighbours<2>, dim3(grid_for(n)), dim3(kBlock), 0, H->stream, n, d_keys, dm,
                       H->slots.as<HSlot<2>>(), H->mask(), d_nbr);
  check_launch();
  return MG_OK;
  MG_API_END
}

mg_status_t mg_hash_rebuild(mg_hash_t H) {
  MG_API_BEGIN
  MG_REQUIRE(H != nullptr, "mg_hash_rebuild: handle is NULL");
  H->rehash(H->capacity_for(H->n_live, 16));
  MG_HIP(hipStreamSynchronize(H->stream));
  return MG_OK;
  MG_API_END
}

mg_status_t mg_hash_info(mg_hash_t H, int64_t* size, int64_t* deleted, int64_t* capacity) {
  MG_API_BEGIN
  MG_REQUIRE(H != nullptr, "mg_hash_info: handle is NULL");
  if (size) *size = H->n_live;
  if (deleted) *deleted = H->n_deleted;
  if (capacity) *capacity = H->cap;
  return MG_OK;
  MG_API_END
}

mg_status_t mg_op_morton128(int64_t n, const int64_t* d_ijk, uint64_t* d_keys, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(n >= 0, "mg_op_morton128: n must be >= 0");
  if (n == 0) return MG_OK;
  MG_REQUIRE(d_ijk && d_keys && aligned8(d_ijk) && aligned8(d_keys), "mg_op_morton128: NULL or misaligned argument");
  hipLaunchKernelGGL(k_morton128, dim3(grid_for(n)), dim3(kBlock), 0, (hipStream_t)stream, n, d_ijk, d_keys);
  check_launch();
  return MG_OK;
  MG_API_END
}

mg_status_t mg_op_hash(int64_t n, int32_t key_words, const uint64_t* d_keys, uint64_t* d_hash, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(n >= 0, "mg_op_hash: n must be >= 0");
  MG_REQUIRE(key_words == 1 || key_words == 2, "mg_op_hash: key_words must be 1 or 2");
  if (n == 0) return MG_OK;
  MG_REQUIRE(d_keys && d_hash && aligned8(d_keys) && aligned8(d_hash), "mg_op_hash: NULL or misaligned argument");
  if (key_words == 1)
    hipLaunchKernelGGL((k_hash_values<1>), dim3(grid_for(n)), dim3(kBlock), 0, (hipStream_t)stream, n, d_keys, d_hash);
  else
    hipLaunchKernelGGL((k_hash_values<2>), dim3(grid_for(n)), dim3(kBlock), 0, (hipStream_t)stream, n, d_keys, d_hash);
  check_launch();
  return MG_OK;
  MG_API_END
}

}  // extern "C"

// C ABI: level build, solve (plain FP64 and FP32-in-FP64 defect correction),
// residual norms and kernel-level entry points.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>

#include "level.h"

namespace mg {

namespace {
thread_local std::string g_error;
}
void set_error(const std::string& msg) { g_error = msg; }
const char* get_error() { return g_error.c_str(); }

// Blocks released by level arenas, kept per device for the next builds (a
// solver that rebuilds its levels every step then allocates nothing new);
// at most kCacheBytes per device, the rest is freed.
namespace {
constexpr size_t kCacheBytes = size_t(8) << 30;
struct BlockCache {
  std::mutex mu;
  std::vector<std::multimap<size_t, void*>> free;   // [device] size -> block
  std::vector<size_t> held;
};
BlockCache& block_cache() {
  static BlockCache* c = new BlockCache();   // never destroyed: blocks live until the process ends
  return *c;
}
// a cached block of at least b and at most 2b bytes, else a new one
void* cached_malloc(int dev, size_t b) {
  {
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    if ((int)c.free.size() > dev) {
      auto it = c.free[dev].lower_bound(b);
      if (it != c.free[dev].end() && it->first <= 2 * b) {
        void* p = it->second;
        c.held[dev] -= it->first;
        c.free[dev].erase(it);
        return p;
      }
    }
  }
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, b);
  if (e == hipErrorOutOfMemory) {   // give the cached blocks back and try once more
    (void)hipGetLastError();
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    if ((int)c.free.size() > dev) {
      for (auto& kv : c.free[dev]) (void)hipFree(kv.second);
      c.free[dev].clear();
      c.held[dev] = 0;
    }
    MG_HIP(hipMalloc(&p, b));
  } else {
    MG_HIP(e);
  }
  return p;
}
}  // namespace

void* DevArena::get(size_t b) {
  if (device < 0) MG_HIP(hipGetDevice(&device));
  b = (b + kAlign - 1) & ~(kAlign - 1);
  if (b >= kAlone) {
    const size_t rb = (b + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);   // 2 MiB granules
    void* p = cached_malloc(device, rb);
    blocks.push_back({p, rb});
    return p;
  }
  if (b > left) {
    void* p = cached_malloc(device, kChunk);
    blocks.push_back({p, kChunk});
    cur = static_cast<char*>(p);
    left = kChunk;
  }
  void* p = cur;
  cur += b;
  left -= b;
  return p;
}

void DevArena::release() noexcept {
  if (!blocks.empty()) {
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();   // no kernel still uses a block (what hipFree would wait for)
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    if ((int)c.free.size() <= device) {
      c.free.resize(device + 1);
      c.held.resize(device + 1, 0);
    }
    for (const Block& k : blocks) {
      if (c.held[device] + k.bytes <= kCacheBytes) {
        c.free[device].emplace(k.bytes, k.p);
        c.held[device] += k.bytes;
      } else {
        (void)hipFree(k.p);
      }
    }
    if (prev >= 0) (void)hipSetDevice(prev);
  }
  blocks.clear();
  cur = nullptr;
  left = 0;
}

DevArena*& current_arena() {
  thread_local DevArena* a = nullptr;
  return a;
}
DevArena*& current_scratch_arena() {
  thread_local DevArena* a = nullptr;
  return a;
}

void prepare_scratch_pool() {
  static std::mutex mu;
  static std::vector<bool> done;
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)done.size() <= dev) done.resize(dev + 1, false);
  if (done[dev]) return;
  hipMemPool_t pool;
  MG_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t keep = uint64_t(1) << 30;   // bytes the pool may hold across synchronisations
  MG_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  done[dev] = true;
}

}  // namespace mg

using namespace mg;

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// ---------------------------------------------------------------------------
// Static device scratch for the entry point that allocates nothing
// (mg_op_resid_restrict_noalloc): the per-workgroup norm partials, one f64
// per workgroup, at most kScratchDoubles of them (4 MiB, enough for n <=
// 1024).  Every GPU the library runs on holds its own copy until the process
// ends; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device, taken once per device.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kScratchDoubles = int64_t(1) << 19;
__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // per device ordinal, NULL until first use

double* scratch_for_current_device() {
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    MG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    MG_REQUIRE(p != nullptr, "static scratch: hipGetSymbolAddress returned NULL");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace


extern "C" {

const char* mg_last_error(void) { return get_error(); }

mg_status_t mg_build_level(const mg_level_desc_t* desc, mg_level_t* out) {
  MG_API_BEGIN
  MG_REQUIRE(out != nullptr, "mg_build_level: out is NULL");
  *out = nullptr;
  MG_REQUIRE(desc != nullptr, "mg_build_level: desc is NULL");
  std::unique_ptr<mg_level_s> L(new mg_level_s());
  L->build(*desc);
  *out = L.release();
  return MG_OK;
  MG_API_END
}

void mg_destroy_level(mg_level_t L) { delete L; }

mg_status_t mg_solve(mg_level_t L, const double* d_rho, double rho_mean, double four_pi_G,
                     const double* d_phi_parent, double* d_phi, double tol, int32_t max_cycles,
                     mg_solve_info_t* info) {
  MG_API_BEGIN
  MG_REQUIRE(L != nullptr, "mg_solve: level handle is NULL");
  MG_REQUIRE(d_rho != nullptr && d_phi != nullptr, "mg_solve: d_rho and d_phi must be non-NULL");
  MG_REQUIRE(aligned16(d_rho) && aligned16(d_phi) && aligned16(d_phi_parent),
             "mg_solve: field arrays must be 16-byte aligned");
  MG_REQUIRE(std::isfinite(four_pi_G) && four_pi_G != 0.0, "mg_solve: four_pi_G must be finite and non-zero");
  MG_REQUIRE(tol > 0.0 && std::isfinite(tol), "mg_solve: tol must be positive");
  MG_REQUIRE(max_cycles >= 0, "mg_solve: max_cycles must be >= 0");
  mg_solve_info_t tmp{};
  mg_status_t st = L->solve(d_rho, rho_mean, four_pi_G, d_phi_parent, d_phi, tol, max_cycles, tmp);
  if (info) *info = tmp;
  return st;
  MG_API_END
}

mg_status_t mg_solve_chain(const mg_level_t* levels, int32_t n_levels, const double* const* d_rho,
                           double rho_mean, double four_pi_G, double* const* d_phi, double tol,
                           int32_t max_cycles, int32_t base_fft, mg_solve_info_t* infos) {
  MG_API_BEGIN
  MG_REQUIRE(levels != nullptr && d_rho != nullptr && d_phi != nullptr, "mg_solve_chain: NULL argument");
  MG_REQUIRE(n_levels >= 1, "mg_solve_chain: n_levels must be >= 1");
  for (int32_t i = 0; i < n_levels; ++i) {
    const mg_level_t L = levels[i];
    MG_REQUIRE(L != nullptr, "mg_solve_chain: a level handle is NULL");
    MG_REQUIRE(L->desc.level == i, "mg_solve_chain: levels[i] must be a level-i handle");
    MG_REQUIRE(i == 0 || L->desc.parent == levels[i - 1], "mg_solve_chain: levels[i] must have parent levels[i-1]");
    MG_REQUIRE(d_rho[i] != nullptr && d_phi[i] != nullptr, "mg_solve_chain: a density or potential is NULL");
    MG_REQUIRE(aligned16(d_rho[i]) && aligned16(d_phi[i]), "mg_solve_chain: field arrays must be 16-byte aligned");
  }
  MG_REQUIRE(std::isfinite(four_pi_G) && four_pi_G != 0.0, "mg_solve_chain: four_pi_G must be finite and non-zero");
  MG_REQUIRE(tol > 0.0 && std::isfinite(tol), "mg_solve_chain: tol must be positive");
  MG_REQUIRE(max_cycles >= 0, "mg_solve_chain: max_cycles must be >= 0");
  mg_status_t worst = MG_OK;
  double mean = rho_mean;
  for (int32_t i = 0; i < n_levels; ++i) {
    mg_solve_info_t tmp{};
    const mg_status_t st =
        (i == 0 && base_fft)
            ? levels[0]->fft_solve(d_rho[0], mean, four_pi_G, d_phi[0], tmp)
            : levels[i]->solve(d_rho[i], mean, four_pi_G, i == 0 ? nullptr : d_phi[i - 1], d_phi[i], tol,
                               max_cycles, tmp);
    if (infos) infos[i] = tmp;
    if (st < 0) return st;
    if (st == MG_NOT_CONVERGED) worst = MG_NOT_CONVERGED;
    if (i == 0) mean = tmp.rho_mean;   // the base level's mean serves every level
  }
  return worst;
  MG_API_END
}

mg_status_t mg_residual_norm(mg_level_t L, const double* d_rho, double rho_mean, double four_pi_G,
                             const double* d_phi_parent, const double* d_phi, double* res_norm,
                             double* rhs_norm) {
  MG_API_BEGIN
  MG_REQUIRE(L != nullptr, "mg_residual_norm: level handle is NULL");
  MG_REQUIRE(d_rho && d_phi && res_norm && rhs_norm, "mg_residual_norm: NULL argument");
  MG_REQUIRE(aligned16(d_rho) && aligned16(d_phi) && aligned16(d_phi_parent),
             "mg_residual_norm: field arrays must be 16-byte aligned");
  MG_REQUIRE(std::isfinite(four_pi_G), "mg_residual_norm: four_pi_G must be finite");
  L->residual_norm(d_rho, rho_mean, four_pi_G, d_phi_parent, d_phi, *res_norm, *rhs_norm);
  return MG_OK;
  MG_API_END
}

mg_status_t mg_fft_solve(mg_level_t L, const double* d_rho, double rho_mean, double four_pi_G, double* d_phi,
                         mg_solve_info_t* info) {
  MG_API_BEGIN
  MG_REQUIRE(L != nullptr, "mg_fft_solve: level handle is NULL");
  MG_REQUIRE(d_rho && d_phi, "mg_fft_solve: NULL argument");
  MG_REQUIRE(aligned16(d_rho) && aligned16(d_phi), "mg_fft_solve: field arrays must be 16-byte aligned");
  MG_REQUIRE(std::isfinite(four_pi_G), "mg_fft_solve: four_pi_G must be finite");
  mg_solve_info_t tmp{};
  const mg_status_t st = L->fft_solve(d_rho, rho_mean, four_pi_G, d_phi, tmp);
  if (info) *info = tmp;
  return st;
  MG_API_END
}

mg_status_t mg_level_smooth(mg_level_t L, const double* d_rho, double rho_mean, double four_pi_G,
                            const double* d_phi_parent, double* d_phi, int32_t n_sweeps) {
  MG_API_BEGIN
  MG_REQUIRE(L != nullptr, "mg_level_smooth: level handle is NULL");
  MG_REQUIRE(d_rho && d_phi, "mg_level_smooth: NULL argument");
  MG_REQUIRE(aligned16(d_rho) && aligned16(d_phi) && aligned16(d_phi_parent),
             "mg_level_smooth: field arrays must be 16-byte aligned");
  MG_REQUIRE(std::isfinite(four_pi_G), "mg_level_smooth: four_pi_G must be finite");
  MG_REQUIRE(n_sweeps >= 0, "mg_level_smooth: n_sweeps must be >= 0");
  L->smooth(d_rho, rho_mean, four_pi_G, d_phi_parent, d_phi, n_sweeps);
  return MG_OK;
  MG_API_END
}

mg_status_t mg_force(mg_level_t L, const double* d_phi_parent, const double* d_phi, double* d_force) {
  MG_API_BEGIN
  MG_REQUIRE(L != nullptr, "mg_force: level handle is NULL");
  MG_REQUIRE(d_phi != nullptr && d_force != nullptr, "mg_force: d_phi and d_force must be non-NULL");
  MG_REQUIRE(aligned16(d_phi) && aligned16(d_force) && aligned16(d_phi_parent),
             "mg_force: field arrays must be 16-byte aligned");
  L->force(d_phi_parent, d_phi, d_force);
  return MG_OK;
  MG_API_END
}

mg_status_t mg_get_neighbors(mg_level_t L, int32_t* d_nbr) {
  MG_API_BEGIN
  MG_REQUIRE(L != nullptr && d_nbr != nullptr, "mg_get_neighbors: NULL argument");
  L->get_neighbors(d_nbr);
  return MG_OK;
  MG_API_END
}

mg_status_t mg_hierarchy_info(mg_level_t L, int32_t* n_levels, int64_t* h_active_cells, int32_t capacity) {
  MG_API_BEGIN
  MG_REQUIRE(L != nullptr && n_levels != nullptr, "mg_hierarchy_info: NULL argument");
  const std::vector<int64_t> act = L->active_cells();
  *n_levels = (int32_t)act.size();
  if (h_active_cells) {
    MG_REQUIRE(capacity >= (int32_t)act.size(), "mg_hierarchy_info: capacity too small");
    std::copy(act.begin(), act.end(), h_active_cells);
  }
  return MG_OK;
  MG_API_END
}

// ---------------------------------------------------------------------------
// kernel-level entry points (full periodic grids)
// ---------------------------------------------------------------------------
static void check_grid(int32_t n, int32_t dtype, int32_t min_n, const char* who) {
  MG_REQUIRE(is_pow2(n) && n >= min_n && n <= 4096, std::string(who) + ": n must be a power of two in [" +
                                                        std::to_string(min_n) + ", 4096]");
  MG_REQUIRE(dtype == 0 || dtype == 1, std::string(who) + ": dtype must be 0 (f64) or 1 (f32)");
}

mg_status_t mg_op_smooth(int32_t n, double h, int32_t dtype, void* d_phi, const void* d_b, int32_t n_sweeps,
                         void* d_work, void* stream) {
  MG_API_BEGIN
  check_grid(n, dtype, 4, "mg_op_smooth");
  MG_REQUIRE(d_phi && d_b && n_sweeps >= 0 && h > 0, "mg_op_smooth: bad argument");
  MG_REQUIRE(aligned16(d_phi) && aligned16(d_b) && aligned16(d_work), "mg_op_smooth: arrays must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const size_t cells = (size_t)n * n * n;
  const size_t es = dtype == 0 ? sizeof(double) : sizeof(float);
  // scratch for the ping-pong tiled sweep: the caller's, or one freed after the stream drains
  DevBuf own(d_work == nullptr && tiled_smoother(n) && n_sweeps > 0 ? cells * es : 0);
  void* work = d_work ? d_work : own.p;
  if (dtype == 0) u_smooth<double>(n, h, (double*)d_phi, (const double*)d_b, n_sweeps, s, (double*)work);
  else u_smooth<float>(n, h, (float*)d_phi, (const float*)d_b, n_sweeps, s, (float*)work);
  if (own.p) MG_HIP(hipStreamSynchronize(s));
  return MG_OK;
  MG_API_END
}

mg_status_t mg_op_force(int32_t n, double h, const double* d_phi, double* d_force, void* stream) {
  MG_API_BEGIN
  check_grid(n, 0, 4, "mg_op_force");
  MG_REQUIRE(d_phi && d_force && h > 0, "mg_op_force: bad argument");
  MG_REQUIRE(aligned16(d_phi) && aligned16(d_force), "mg_op_force: arrays must be 16-byte aligned");
  u_force(n, h, d_phi, d_force, (hipStream_t)stream);
  return MG_OK;
  MG_API_END
}

mg_status_t mg_op_resid_restrict(int32_t n, double h, int32_t dtype, const void* d_phi, const void* d_b,
                                 void* d_bc, double* d_norm2, void* stream) {
  MG_API_BEGIN
  check_grid(n, dtype, 4, "mg_op_resid_restrict");
  MG_REQUIRE(d_phi && d_b && h > 0, "mg_op_resid_restrict: bad argument");
  MG_REQUIRE(aligned16(d_phi) && aligned16(d_b) && aligned16(d_bc), "mg_op_resid_restrict: arrays must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n_oct = (int64_t)(n / 2) * (n / 2) * (n / 2);
  DevBuf parts(partial_count(n_oct, kReduceBlock) * sizeof(double));   // >= tiled_sweep_blocks(n)
  int64_t np = 0;
  if (dtype == 0)
    np = u_resid_restrict<double>(n, h, (const double*)d_phi, (const double*)d_b, (double*)d_bc, parts.as<double>(), s);
  else
    np = u_resid_restrict<float>(n, h, (const float*)d_phi, (const float*)d_b, (float*)d_bc, parts.as<double>(), s);
  if (d_norm2) reduce_final(parts.as<double>(), np, 1.0, d_norm2, 0, s);
  MG_HIP(hipStreamSynchronize(s));
  return MG_OK;
  MG_API_END
}

mg_status_t mg_op_resid_restrict_noalloc(int32_t n, double h, int32_t dtype, const void* d_phi, const void* d_b,
                                         void* d_bc, double* d_norm2, void* stream) {
  MG_API_BEGIN
  check_grid(n, dtype, 4, "mg_op_resid_restrict_noalloc");
  MG_REQUIRE(d_phi && d_b && h > 0, "mg_op_resid_restrict_noalloc: bad argument");
  MG_REQUIRE(aligned16(d_phi) && aligned16(d_b) && aligned16(d_bc),
             "mg_op_resid_restrict_noalloc: arrays must be 16-byte aligned");
  const int64_t n_oct = (int64_t)(n / 2) * (n / 2) * (n / 2);
  // the partial count u_resid_restrict writes is at most this (the same bound
  // mg_op_resid_restrict allocates for)
  MG_REQUIRE(partial_count(n_oct, kReduceBlock) <= kScratchDoubles,
             "mg_op_resid_restrict_noalloc: n exceeds the static scratch (n <= 1024)");
  hipStream_t s = (hipStream_t)stream;
  double* parts = d_norm2 ? scratch_for_current_device() : nullptr;
  int64_t np = 0;
  if (dtype == 0)
    np = u_resid_restrict<double>(n, h, (const double*)d_phi, (const double*)d_b, (double*)d_bc, parts, s);
  else
    np = u_resid_restrict<float>(n, h, (const float*)d_phi, (const float*)d_b, (float*)d_bc, parts, s);
  if (d_norm2) reduce_final(parts, np, 1.0, d_norm2, 0, s);
  return MG_OK;
  MG_API_END
}

mg_status_t mg_op_prolong(int32_t n, int32_t dtype, const void* d_ec, void* d_e, void* stream) {
  MG_API_BEGIN
  check_grid(n, dtype, 4, "mg_op_prolong");
  MG_REQUIRE(d_ec && d_e, "mg_op_prolong: NULL argument");
  MG_REQUIRE(aligned16(d_ec) && aligned16(d_e), "mg_op_prolong: arrays must be 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (dtype == 0) u_prolong<double>(n, (const double*)d_ec, (double*)d_e, s);
  else u_prolong<float>(n, (const float*)d_ec, (float*)d_e, s);
  return MG_OK;
  MG_API_END
}

mg_status_t mg_op_coarse_solve(int32_t n, double h, int32_t dtype, const void* d_b, void* d_e, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(n == 2 || n == 4 || n == 8, "mg_op_coarse_solve: n must be 2, 4 or 8");
  MG_REQUIRE(dtype == 0 || dtype == 1, "mg_op_coarse_solve: bad dtype");
  MG_REQUIRE(d_b && d_e && h > 0, "mg_op_coarse_solve: bad argument");
  hipStream_t s = (hipStream_t)stream;
  std::vector<double> G = coarse_pinv(n, h);
  const int N = n * n * n;
  DevBuf dG;
  if (dtype == 0) {
    dG.alloc(G.size() * sizeof(double));
    MG_HIP(hipMemcpyAsync(dG.p, G.data(), G.size() * sizeof(double), hipMemcpyHostToDevice, s));
    u_coarse_solve<double>(n, dG.as<double>(), (const double*)d_b, (double*)d_e, s);
  } else {
    std::vector<float> Gf(G.begin(), G.end());
    dG.alloc(Gf.size() * sizeof(float));
    MG_HIP(hipMemcpyAsync(dG.p, Gf.data(), Gf.size() * sizeof(float), hipMemcpyHostToDevice, s));
    u_coarse_solve<float>(n, dG.as<float>(), (const float*)d_b, (float*)d_e, s);
  }
  (void)N;
  MG_HIP(hipStreamSynchronize(s));
  return MG_OK;
  MG_API_END
}

static mg_status_t layout_call(int32_t n, const double* in, double* out, void* stream, bool to_oct, const char* who) {
  MG_API_BEGIN
  MG_REQUIRE(is_pow2(n) && n >= 2 && n <= 4096, std::string(who) + ": n must be a power of two in [2, 4096]");
  MG_REQUIRE(in && out, std::string(who) + ": NULL argument");
  MG_REQUIRE(aligned16(in) && aligned16(out), std::string(who) + ": arrays must be 16-byte aligned");
  const uintptr_t bytes = (uintptr_t)n * n * n * sizeof(double);
  const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  MG_REQUIRE(a + bytes <= b || b + bytes <= a, std::string(who) + ": input and output overlap");
  u_layout(n, to_oct, in, out, (hipStream_t)stream);
  return MG_OK;
  MG_API_END
}

mg_status_t mg_dense_to_oct(int32_t n, const double* d_dense, double* d_oct, void* stream) {
  return layout_call(n, d_dense, d_oct, stream, true, "mg_dense_to_oct");
}

mg_status_t mg_oct_to_dense(int32_t n, const double* d_oct, double* d_dense, void* stream) {
  return layout_call(n, d_oct, d_dense, stream, false, "mg_oct_to_dense");
}

mg_status_t mg_op_morton(int64_t n, const int32_t* d_ijk, uint64_t* d_keys, void* stream) {
  MG_API_BEGIN
  MG_REQUIRE(n >= 0, "mg_op_morton: n must be >= 0");
  if (n == 0) return MG_OK;
  MG_REQUIRE(d_ijk && d_keys, "mg_op_morton: NULL argument");
  morton_keys(n, d_ijk, d_keys, (hipStream_t)stream);
  return MG_OK;
  MG_API_END
}

}  // extern "C"

// Level build and the solve drivers (host side).
//
// V-cycle of the correction scheme (algorithm "GPU-accelerated V-cycle at AMR
// level l"): nu_pre red-black sweeps, fused residual + restriction, recursive
// cycle on the coarse error equation from a zero guess, prolongation +
// correction, nu_post red-black sweeps.  The coarse operator is the 7-point
// stencil re-discretised at spacing 2h.  Convergence is checked after every
// cycle on ||f - L phi||_2 / ||f||_2, read back as one f64.
//
// Periodic levels use the arithmetic hierarchy n, n/2, ..., 4 with an exact
// pseudo-inverse solve on 4^3.  Refined levels use the father-cell hierarchy:
// coarse level m+1 holds the father cells of level m's octs (grouped in their
// octs, other cells masked to 0), down to at most coarsest_oct_capacity()
// octs, which are relaxed by red-black sweeps inside one workgroup.
#include <algorithm>
#include <cstring>

#include "level.h"

#include <type_traits>

using namespace mg;

mg_level_s::~mg_level_s() {
  if (hp) (void)hipHostFree(hp);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  for (hipEvent_t e : evq)
    if (e) (void)hipEventDestroy(e);
}

void mg_level_s::build(const mg_level_desc_t& d) {
  MG_REQUIRE(is_pow2(d.base_n) && d.base_n >= 8 && d.base_n <= 4096,
             "mg_build_level: base_n must be a power of two in [8, 4096]");
  MG_REQUIRE(d.level >= 0 && d.level <= 30, "mg_build_level: level must be in [0, 30]");
  const int64_t ncell = (int64_t)d.base_n << d.level;
  MG_REQUIRE(ncell / 2 <= (int64_t(1) << 31),
             "mg_build_level: oct coordinates exceed the int32 range (base_n * 2^(level-1) > 2^31)");
  MG_REQUIRE(d.nu_pre >= 0 && d.nu_pre <= 16 && d.nu_post >= 0 && d.nu_post <= 16 && d.nu_pre + d.nu_post > 0,
             "mg_build_level: nu_pre/nu_post must be in [0, 16] and not both 0");
  MG_REQUIRE(d.precision == MG_PREC_FP64 || d.precision == MG_PREC_MIXED, "mg_build_level: bad precision");
  MG_REQUIRE(d.load_factor > 0.0 && d.load_factor <= 0.9, "mg_build_level: load_factor must be in (0, 0.9]");
  MG_REQUIRE(d.coarsest_n == 0 || d.coarsest_n == 2 || d.coarsest_n == 4 || d.coarsest_n == 8,
             "mg_build_level: coarsest_n must be 2, 4 or 8 (0 selects 4)");
  MG_REQUIRE(d.brick_shift >= 0 && d.brick_shift <= 8, "mg_build_level: brick_shift must be in [0, 8]");
  if (d.level == 0) {
    MG_REQUIRE(d.d_oct_ijk == nullptr && d.parent == nullptr,
               "mg_build_level: level 0 takes no oct list and no parent");
    const int64_t no = d.base_n / 2;
    MG_REQUIRE(d.n_oct == no * no * no, "mg_build_level: level 0 needs n_oct = (base_n/2)^3");
  } else {
    MG_REQUIRE(d.d_oct_ijk != nullptr, "mg_build_level: refined level needs d_oct_ijk");
    MG_REQUIRE(d.parent != nullptr, "mg_build_level: refined level needs a parent handle");
    MG_REQUIRE(d.parent->desc.level == d.level - 1 && d.parent->desc.base_n == d.base_n,
               "mg_build_level: parent must be level-1 with the same base_n");
    MG_REQUIRE(d.n_oct >= 1 && d.n_oct <= (int64_t(1) << 28), "mg_build_level: n_oct must be in [1, 2^28]");
  }
  desc = d;
  coarsest_n = d.coarsest_n == 0 ? 4 : d.coarsest_n;
  MG_REQUIRE(coarsest_n <= d.base_n, "mg_build_level: coarsest_n must not exceed base_n");
  stream = (hipStream_t)d.stream;
  periodic = (d.level == 0);
  mixed = (d.precision == MG_PREC_MIXED);
  n = ncell <= (int64_t(1) << 30) ? (int)ncell : 0;   // cells per dimension (read on periodic levels)
  h = 1.0 / (double)ncell;
  n_oct = d.n_oct;
  n_cells = 8 * n_oct;

  MG_HIP(hipHostMalloc((void**)&hp, 8 * sizeof(double), hipHostMallocDefault));
  MG_HIP(hipEventCreate(&ev0));
  MG_HIP(hipEventCreate(&ev1));
  for (hipEvent_t& e : evq) MG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  scalars.alloc(8 * sizeof(double));
  f.alloc(n_cells * sizeof(double));
  n_partials = partial_count(n_cells, kReduceBlock);
  partials.alloc(n_partials * sizeof(double));
  if (periodic) build_uniform();
  else build_refined();
  MG_HIP(hipStreamSynchronize(stream));
}

void mg_level_s::build_uniform() {
  un.clear();
  for (int m = n; m >= coarsest_n; m /= 2) un.push_back(m);
  const int M = (int)un.size();
  for (int p = 0; p < 2; ++p) {
    ue[p].clear();
    ub[p].clear();
    ut[p].clear();
    ue[p].resize(M);
    ub[p].resize(M);
    ut[p].resize(M);
  }
  const int p = mixed ? 1 : 0;
  const size_t es = mixed ? sizeof(float) : sizeof(double);
  for (int m = 0; m < M; ++m) {
    const size_t cells = (size_t)un[m] * un[m] * un[m];
    if (m > 0 || mixed) {
      ue[p][m].alloc(cells * es);
      ub[p][m].alloc(cells * es);
    }
    if (tiled_smoother(un[m])) ut[p][m].alloc(cells * es);
  }
  const double hM = h * (double)(n / un[M - 1]);
  std::vector<double> Gd = coarse_pinv(un[M - 1], hM);
  if (mixed) {
    std::vector<float> Gf(Gd.begin(), Gd.end());
    G[1].alloc(Gf.size() * sizeof(float));
    MG_HIP(hipMemcpy(G[1].p, Gf.data(), Gf.size() * sizeof(float), hipMemcpyHostToDevice));
  } else {
    G[0].alloc(Gd.size() * sizeof(double));
    MG_HIP(hipMemcpy(G[0].p, Gd.data(), Gd.size() * sizeof(double), hipMemcpyHostToDevice));
  }
}

// Key frame of a refined level (see level.h): per axis, the octs' coordinates
// are taken round the periodic circle of the level's extent, the largest gap
// between them found, and the frame placed one oct before the first
// coordinate after that gap, rounded down to the largest power of two (up to
// 2^20) that still leaves every relative coordinate in [1, 2^21 - 2].
// Returns the relative coordinates (int32, [n][3]) for the device.
static std::vector<int32_t> key_frame(const std::vector<int32_t>& ijk, int64_t n_true, int64_t (&frame)[3]) {
  const int64_t kSpace = int64_t(1) << 21;
  const int64_t n = (int64_t)ijk.size() / 3;
  std::vector<int32_t> rel(ijk.size());
  for (int a = 0; a < 3; ++a) {
    std::vector<int64_t> u(n);
    for (int64_t i = 0; i < n; ++i) {
      u[i] = ijk[3 * i + a];
      MG_REQUIRE(u[i] >= 0 && u[i] < n_true, "mg_build_level: oct coordinate outside [0, base_n*2^level/2)");
    }
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    // the largest gap on the circle ends at `start`
    int64_t best_gap = u.front() + n_true - u.back(), start = u.front();
    for (size_t k = 1; k < u.size(); ++k)
      if (u[k] - u[k - 1] > best_gap) {
        best_gap = u[k] - u[k - 1];
        start = u[k];
      }
    const int64_t span = (u.size() == 1) ? 0 : n_true - best_gap;   // last - first round the circle
    MG_REQUIRE(span <= kSpace - 4,
               "mg_build_level: on a level deeper than 2^21 octs per axis the octs must lie within 2^21 - 4 "
               "consecutive octs along each axis");
    const int64_t origin = (start - 1 + n_true) % n_true;
    int64_t f = origin;
    for (int al = 20; al >= 0; --al) {
      const int64_t lo = origin & ((int64_t(1) << al) - 1);
      if (lo + span + 2 <= kSpace - 2) {
        f = origin - lo;
        break;
      }
    }
    frame[a] = f;
    for (int64_t i = 0; i < n; ++i) rel[3 * i + a] = (int32_t)(((int64_t)ijk[3 * i + a] - f + n_true) % n_true);
  }
  return rel;
}

void mg_level_s::build_refined() {
  const int64_t n_true = ((int64_t)desc.base_n << desc.level) / 2;   // octs per dimension of the level's extent
  const int64_t kSpace = int64_t(1) << 21;
  const int32_t* ijk = desc.d_oct_ijk;
  // the level's buffers from its arena, the steps' scratch from one arena for
  // the whole build (handed back once the build's work is done)
  DevArena scratch_arena;
  ArenaScope arena_scope(&arena, &scratch_arena);
  DevBuf rel_dev;
  if (n_true <= kSpace) {
    key_dim = n_true;
  } else {
    std::vector<int32_t> hc((size_t)n_oct * 3);
    MG_HIP(hipMemcpyAsync(hc.data(), desc.d_oct_ijk, hc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    MG_HIP(hipStreamSynchronize(stream));
    const std::vector<int32_t> rel = key_frame(hc, n_true, frame);
    rel_dev.scratch(rel.size() * sizeof(int32_t), stream);
    MG_HIP(hipMemcpyAsync(rel_dev.p, rel.data(), rel.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    MG_HIP(hipStreamSynchronize(stream));
    ijk = rel_dev.as<int32_t>();
    key_dim = kSpace;
  }
  const int n_dim = (int)key_dim;   // octs per dimension of the key space
  ol.clear();
  ol.emplace_back();
  OctLevel& L0 = ol[0];
  L0.n_oct = n_oct;
  L0.n_dim = n_dim;
  L0.h = h;
  L0.n_active = n_cells;
  L0.keys.alloc(n_oct * sizeof(uint64_t));
  DevBuf flag;
  flag.scratch(sizeof(int), stream);
  MG_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), stream));
  oct_validate(n_oct, ijk, n_dim, flag.as<int>(), stream);
  morton_keys(n_oct, ijk, L0.keys.as<uint64_t>(), stream);

  // hash table at the requested load factor
  int64_t cap = 1;
  while ((double)cap * desc.load_factor < (double)n_oct) cap <<= 1;
  hash.capacity = cap;
  hash.slots.alloc(cap * hash_slot_bytes());
  hash_build(n_oct, L0.keys.as<uint64_t>(), hash.slots.p, cap, flag.as<int>(), stream);
  int hflag = 0;
  MG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  MG_HIP(hipStreamSynchronize(stream));
  MG_REQUIRE(!(hflag & 1), "mg_build_level: oct coordinate outside [0, base_n*2^level/2)");
  MG_REQUIRE(!(hflag & 2), "mg_build_level: duplicate oct coordinates");
  if (hflag & 4) {
    set_error("mg_build_level: hash table full");
    throw Fail{MG_ERR_TABLE};
  }

  // neighbour cache and ghost faces
  L0.nbr.alloc(n_oct * 6 * sizeof(int32_t));
  DevBuf missing, first;
  missing.scratch(n_oct * sizeof(int32_t), stream);
  first.scratch(n_oct * sizeof(int32_t), stream);
  nbr_from_hash(n_oct, L0.keys.as<uint64_t>(), n_dim, hash.slots.p, cap, L0.nbr.as<int32_t>(),
                missing.as<int32_t>(), stream);
  exclusive_scan_i32(n_oct, missing.as<int32_t>(), first.as<int32_t>(), stream);
  int32_t last[2] = {0, 0};
  MG_HIP(hipMemcpyAsync(&last[0], first.as<int32_t>() + (n_oct - 1), sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  MG_HIP(hipMemcpyAsync(&last[1], missing.as<int32_t>() + (n_oct - 1), sizeof(int32_t), hipMemcpyDeviceToHost,
                        stream));
  MG_HIP(hipStreamSynchronize(stream));
  n_ghost = (int64_t)last[0] + last[1];
  ghost_idx.alloc(std::max<int64_t>(n_ghost, 1) * 32 * sizeof(int32_t));
  ghost_val.alloc(std::max<int64_t>(n_ghost, 1) * 4 * sizeof(double));
  const mg_level_s* P = desc.parent;
  // this level's relative oct coordinate + shift = the parent's relative cell coordinate
  const int64_t pcells = P->periodic ? (int64_t)P->n : 2 * P->key_dim;
  int shift[3];
  for (int a = 0; a < 3; ++a) {
    int64_t sh = frame[a] - 2 * P->frame[a];
    // a parent without a frame wraps at its true extent; in a parent's frame
    // the shift may be negative (the frames are rounded independently), and
    // cells outside the parent's octs are found missing by the lookups
    if (P->periodic || P->key_dim < kSpace) sh = ((sh % pcells) + pcells) % pcells;
    MG_REQUIRE(sh > -pcells && sh < pcells, "mg_build_level: internal error: key frames too far apart");
    shift[a] = (int)sh;
  }
  ghost_stencils(n_oct, L0.keys.as<uint64_t>(), n_dim, first.as<int32_t>(), L0.nbr.as<int32_t>(), P->periodic,
                 P->periodic ? nullptr : P->hash.slots.p, P->periodic ? 0 : P->hash.capacity, (int)pcells, shift,
                 ghost_idx.as<int32_t>(), flag.as<int>(), stream);
  // (the stencils' flag is read with the hierarchy's, below)

  // father-cell hierarchy
  const int cap_octs = coarsest_oct_capacity();
  while ((ol.size() == 1 || ol.back().n_oct > cap_octs) && ol.back().n_dim > 1) {
    OctLevel& F = ol.back();
    OctLevel C;
    C.n_dim = F.n_dim / 2;
    C.h = 2.0 * F.h;
    const int key_bits = std::min(64, 3 * std::max(1, ilog2(C.n_dim)) + 3);
    // the caller's octs come in any order, the coarse levels' keys ascending
    C.n_oct = unique_parent_keys(F.n_oct, F.keys.as<uint64_t>(), C.keys, key_bits, ol.size() > 1, false, stream);
    F.father.alloc(F.n_oct * sizeof(int32_t));
    fathers(F.n_oct, F.keys.as<uint64_t>(), C.keys.as<uint64_t>(), C.n_oct, F.father.as<int32_t>(), flag.as<int>(),
            stream);
    C.nbr.alloc(C.n_oct * 6 * sizeof(int32_t));
    C.nbr27.alloc(C.n_oct * 27 * sizeof(int32_t));
    nbr_sorted(C.n_oct, C.keys.as<uint64_t>(), C.n_dim, C.nbr.as<int32_t>(), C.nbr27.as<int32_t>(), stream);
    C.lsm.alloc(C.n_oct * 8 * sizeof(float));
    coarse_level_set(F.n_oct, F.father.as<int32_t>(), F.lsm.as<float>(), C.n_oct, C.lsm.as<float>(), stream);
    C.mask.alloc(C.n_oct * sizeof(uint8_t));
    if (mixed) {
      C.diag.alloc(C.n_oct * 8 * sizeof(float));
      level_set_operator<float>(C.n_oct, C.nbr.as<int32_t>(), C.lsm.as<float>(), C.mask.as<uint8_t>(),
                                C.diag.as<float>(), stream);
    } else {
      C.diag.alloc(C.n_oct * 8 * sizeof(double));
      level_set_operator<double>(C.n_oct, C.nbr.as<int32_t>(), C.lsm.as<float>(), C.mask.as<uint8_t>(),
                                 C.diag.as<double>(), stream);
    }
    ol.push_back(std::move(C));
  }
  MG_REQUIRE(ol.back().n_oct <= cap_octs, "mg_build_level: could not coarsen the level below the coarsest size");
  {
    // active cells of each coarse level, and the flags of the ghost stencils
    // and fathers, in one read
    DevBuf act;
    act.scratch(ol.size() * sizeof(unsigned long long), stream);
    MG_HIP(hipMemsetAsync(act.p, 0, ol.size() * sizeof(unsigned long long), stream));
    for (size_t m = 0; m < ol.size(); ++m)
      if (ol[m].mask.p) count_active(ol[m].n_oct, ol[m].mask.as<uint8_t>(), act.as<unsigned long long>() + m, stream);
    std::vector<unsigned long long> hact(ol.size(), 0);
    MG_HIP(hipMemcpyAsync(hact.data(), act.p, ol.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
    MG_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, stream));
    MG_HIP(hipStreamSynchronize(stream));
    if (hflag & 8) {
      set_error("mg_build_level: a ghost's coarse interpolation stencil is missing on the parent level "
                "(octs are not properly nested)");
      throw Fail{MG_ERR_NESTING};
    }
    if (hflag & 16) {
      set_error("mg_build_level: internal error: a father oct is missing from the coarse level");
      throw Fail{MG_ERR_HIP};
    }
    for (size_t m = 0; m < ol.size(); ++m)
      if (ol[m].mask.p) ol[m].n_active = (int64_t)hact[m];
  }
  // A level whose cells are all inactive carries no unknowns: its correction,
  // and with it that of every level below, is identically zero.  The
  // hierarchy ends above it, and its new last level is only smoothed (the
  // same arithmetic as before the cut, without the launches that add zero).
  for (size_t m = 1; m < ol.size(); ++m) {
    if (ol[m].n_active == 0) {
      ol.resize(m);
      last_smooth_only = true;
      break;
    }
  }

  // work arrays: coarse levels (and level 0 of the f32 inner cycle)
  const int p = mixed ? 1 : 0;
  const size_t es = mixed ? sizeof(float) : sizeof(double);
  for (size_t m = (mixed ? 0 : 1); m < ol.size(); ++m) {
    const size_t bytes = (size_t)ol[m].n_oct * 8 * es;
    ol[m].e[p].alloc(bytes);
    ol[m].b[p].alloc(bytes);
    MG_HIP(hipMemsetAsync(ol[m].b[p].p, 0, bytes, stream));
    MG_HIP(hipMemsetAsync(ol[m].e[p].p, 0, bytes, stream));
  }
  // the tail: the first coarse level from which all levels' active cells,
  // their values and tables fit one workgroup's LDS
  {
    int64_t below = 0;
    const int64_t n_last = ol.back().n_active;
    for (int m = (int)ol.size() - 1; m >= 1; --m) {
      below += ol[m].n_active;
      if (tail_lds_bytes(below, ol[m].n_active, n_last, es) > tail_lds_limit() ||
          (int)ol.size() - m > kTailMaxLevels)
        break;
      tail_t = m;
    }
    if (tail_t > 0) {
      if (mixed) build_tail<float>(tail_t);
      else build_tail<double>(tail_t);
    }
  }
  // bricks for the LDS-staged sweeps, and the sweeps' ping-pong twins (not on
  // the coarsest level, which is solved in one workgroup, unless the hierarchy
  // was cut and its last level is only smoothed; not on the tail levels)
  const size_t brick_levels = tail_t > 0 ? (size_t)tail_t : ol.size() - (last_smooth_only ? 0 : 1);
  for (size_t m = 0; m < brick_levels; ++m) {
    OctLevel& L = ol[m];
    if (L.n_dim < 4) continue;
    DevBuf bk;
    L.bshift = desc.brick_shift > 0 ? desc.brick_shift - 1
                                 : choose_brick_shift(L.n_oct, L.keys.as<uint64_t>(), L.n_dim, stream);
    L.n_bricks = brick_keys(L.n_oct, L.keys.as<uint64_t>(), m > 0, L.n_dim, L.bshift, bk, stream);
    L.bmap.alloc(L.n_bricks * 216 * sizeof(int32_t));
    brick_map(L.n_bricks, bk.as<uint64_t>(), L.n_dim, L.bshift, m == 0 ? hash.slots.p : nullptr,
              m == 0 ? hash.capacity : 0, L.keys.as<uint64_t>(), L.n_oct, L.bmap.as<int32_t>(), stream);
    if (m + 1 < ol.size()) {   // coarse boxes for the prolongation from the next level
      L.cmap.alloc(L.n_bricks * 125 * sizeof(int32_t));
      brick_cmap(L.n_bricks, bk.as<uint64_t>(), ol[m + 1].n_dim, L.bshift, ol[m + 1].keys.as<uint64_t>(),
                 ol[m + 1].n_oct, L.cmap.as<int32_t>(), stream);
    }
    L.t[p].alloc((size_t)L.n_oct * 8 * es);
    if (m == 0 && p == 1) L.t[0].alloc((size_t)L.n_oct * 8 * sizeof(double));   // f64 sweeps of mg_level_smooth
    if (m == 0) {
      L.n_gentries =
          mg::brick_ghosts(L.n_bricks, L.bmap.as<int32_t>(), L.nbr.as<int32_t>(), L.gfirst, L.gcell, L.gidx, stream);
      L.gpack.alloc(std::max<int64_t>(L.n_gentries, 1) * sizeof(double));
      if (L.n_bricks > n_partials) {   // one norm partial per brick
        n_partials = L.n_bricks;
        partials.alloc(n_partials * sizeof(double));
      }
    }
  }
  MG_HIP(hipStreamSynchronize(stream));
}

// Tables of the tail levels t .. last (host-built from the levels' masks,
// neighbours, diagonals, fathers and coarse 27-neighbourhoods).
template <typename T>
void mg_level_s::build_tail(int t) {
  const int nl = (int)ol.size() - t;
  std::vector<std::vector<uint8_t>> mask(nl);
  std::vector<std::vector<int32_t>> nbr(nl), father(nl), nbr27(nl), idx(nl);
  std::vector<std::vector<T>> diag(nl);
  // every table the tail needs, gathered on the device and read in one copy
  struct Piece {
    const DevBuf* b;
    size_t bytes;
    void* dst;
  };
  std::vector<Piece> pieces;
  const OctLevel& up = ol[t - 1];
  std::vector<int32_t> fup(up.n_oct);
  for (int k = 0; k < nl; ++k) {
    const OctLevel& L = ol[t + k];
    const int64_t no = L.n_oct;
    mask[k].resize(no);
    nbr[k].resize(no * 6);
    diag[k].resize(no * 8);
    pieces.push_back({&L.mask, (size_t)no, mask[k].data()});
    pieces.push_back({&L.nbr, no * 6 * sizeof(int32_t), nbr[k].data()});
    pieces.push_back({&L.diag, no * 8 * sizeof(T), diag[k].data()});
    if (k + 1 < nl) {
      father[k].resize(no);
      pieces.push_back({&L.father, no * sizeof(int32_t), father[k].data()});
    }
    if (k > 0) {
      nbr27[k].resize(no * 27);
      pieces.push_back({&L.nbr27, no * 27 * sizeof(int32_t), nbr27[k].data()});
    }
  }
  pieces.push_back({&up.father, up.n_oct * sizeof(int32_t), fup.data()});
  {
    size_t total_bytes = 0;
    for (const Piece& q : pieces) total_bytes += (q.bytes + 15) & ~size_t(15);
    DevBuf stage;
    stage.scratch(total_bytes, stream);
    size_t off = 0;
    for (const Piece& q : pieces) {
      MG_HIP(hipMemcpyAsync(stage.as<char>() + off, q.b->p, q.bytes, hipMemcpyDeviceToDevice, stream));
      off += (q.bytes + 15) & ~size_t(15);
    }
    std::vector<char> host(total_bytes);
    MG_HIP(hipMemcpyAsync(host.data(), stage.p, total_bytes, hipMemcpyDeviceToHost, stream));
    MG_HIP(hipStreamSynchronize(stream));
    off = 0;
    for (const Piece& q : pieces) {
      std::memcpy(q.dst, host.data() + off, q.bytes);
      off += (q.bytes + 15) & ~size_t(15);
    }
  }
  TailArgs a;
  a.levels = nl;
  a.nu_pre = desc.nu_pre;
  a.nu_post = desc.nu_post;
  a.last_sweeps = last_smooth_only ? desc.nu_pre + desc.nu_post : coarse_sweeps;
  int total = 0;
  std::vector<int32_t> cell0;
  for (int k = 0; k < nl; ++k) {
    const OctLevel& L = ol[t + k];
    const int64_t no = L.n_oct;
    // compact order: red cells, then black, each in oct order
    idx[k].assign(no * 8, -1);
    a.off[k] = total;
    for (int colour = 0; colour < 2; ++colour) {
      for (int64_t o = 0; o < no; ++o)
        for (int c = 0; c < 8; ++c)
          if (((c ^ (c >> 1) ^ (c >> 2)) & 1) == colour && ((mask[k][o] >> c) & 1u)) {
            idx[k][o * 8 + c] = total++;
            if (k == 0) cell0.push_back((int32_t)(o * 8 + c));
          }
      if (colour == 0) a.nred[k] = total - a.off[k];
    }
    a.h2[k] = L.h * L.h;
    a.inv_h2[k] = 1.0 / (L.h * L.h);
  }
  a.off[nl] = total;
  const int nf = a.off[1], nlb = a.off[nl - 1];
  MG_REQUIRE(tail_lds_bytes(total, nf, total - nlb, sizeof(T)) <= tail_lds_limit() && total < 32768,
             "internal: tail larger than planned");
  a.ns = (total + 3) / 4 * 4;
  const size_t blob_bytes = tail_blob_bytes(total, nf, total - nlb, sizeof(T));
  a.blob16 = (int)(blob_bytes / 16);
  std::vector<unsigned char> blob(blob_bytes, 0);
  T* dg = reinterpret_cast<T*>(blob.data());
  int16_t* nb = reinterpret_cast<int16_t*>(dg + total);
  int16_t* kids = nb + 6 * (size_t)total;
  int16_t* par = kids + 8 * (size_t)(total - nf);
  std::fill(nb, nb + 6 * (size_t)total + 8 * (size_t)(total - nf) + 8 * (size_t)nlb, (int16_t)-1);
  for (int k = 0; k < nl; ++k) {
    const int64_t no = ol[t + k].n_oct;
    for (int64_t o = 0; o < no; ++o)
      for (int c = 0; c < 8; ++c) {
        const int i = idx[k][o * 8 + c];
        if (i < 0) continue;
        dg[i] = diag[k][o * 8 + c];
        for (int j = 0; j < 6; ++j) {   // -x, +x, -y, +y, -z, +z
          const int d = j >> 1, side = j & 1;
          const int64_t oo = ((c >> d) & 1) == side ? nbr[k][o * 6 + j] : o;
          nb[(size_t)i * 6 + j] = (int16_t)(oo >= 0 ? idx[k][oo * 8 + (c ^ (1 << d))] : -1);
        }
        if (k + 1 < nl) {   // prolongation sources on the next level
          const int32_t F = father[k][o], O = F >> 3, cf = F & 7;
          for (int jj = 0; jj < 8; ++jj) {
            const int ax = (jj >> 2) & 1, ay = (jj >> 1) & 1, az = jj & 1;
            const int tx = (cf & 1) + ax * ((c & 1) ? 1 : -1), ty = ((cf >> 1) & 1) + ay * ((c & 2) ? 1 : -1),
                      tz = (cf >> 2) + az * ((c & 4) ? 1 : -1);   // in [-1, 2]
            const int q = ((tz + 2) / 2) * 9 + ((ty + 2) / 2) * 3 + (tx + 2) / 2;   // oct offset + 1 per axis
            const int32_t co = nbr27[k + 1][(int64_t)O * 27 + q];
            const int cc = (tx & 1) + 2 * (ty & 1) + 4 * (tz & 1);
            par[(size_t)i * 8 + jj] = (int16_t)(co >= 0 ? idx[k + 1][(int64_t)co * 8 + cc] : -1);
          }
        }
      }
    if (k + 1 < nl) {   // restriction: each oct's 8 cells into its father cell
      for (int64_t o = 0; o < no; ++o) {
        const int F = idx[k + 1][father[k][o]];
        if (F < 0) continue;
        for (int c = 0; c < 8; ++c) kids[(size_t)(F - nf) * 8 + c] = (int16_t)idx[k][o * 8 + c];
      }
    }
  }
  // the level above restricts straight into the compact right-hand side
  for (int32_t& f : fup) f = idx[0][f];
  tail_blob.alloc(blob_bytes);
  tail_b.alloc(std::max<size_t>(nf, 1) * sizeof(T));
  tail_father.alloc(fup.size() * sizeof(int32_t));
  tail_cell.alloc(std::max<size_t>(cell0.size(), 1) * sizeof(int32_t));
  MG_HIP(hipMemcpyAsync(tail_blob.p, blob.data(), blob_bytes, hipMemcpyHostToDevice, stream));
  MG_HIP(hipMemcpyAsync(tail_father.p, fup.data(), fup.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  MG_HIP(hipMemcpyAsync(tail_cell.p, cell0.data(), cell0.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  MG_HIP(hipStreamSynchronize(stream));   // the host vectors are the copies' sources
  tail_args = a;
}

BrickGhosts mg_level_s::brick_ghosts(bool with_values) const {
  BrickGhosts g;
  if (!with_values || ol.empty() || ol[0].n_bricks == 0) return g;
  g.first = ol[0].gfirst.as<int32_t>();
  g.cell = ol[0].gcell.as<int32_t>();
  g.val = ol[0].gpack.as<double>();
  return g;
}

void mg_level_s::read_scalars(int count) {
  MG_HIP(hipMemcpyAsync(hp, scalars.p, count * sizeof(double), hipMemcpyDeviceToHost, stream));
  MG_HIP(hipStreamSynchronize(stream));
}

void mg_level_s::prepare_rhs(const double* rho, double rho_mean, double c, const double* phi_parent) {
  double* sc = scalars.as<double>();
  if (periodic) {
    MG_REQUIRE(phi_parent == nullptr, "periodic level: d_phi_parent must be NULL");
  } else {
    MG_REQUIRE(phi_parent != nullptr, "refined level: d_phi_parent is required");
    MG_REQUIRE(std::isfinite(rho_mean), "refined level: rho_mean must be finite (the base level's mean)");
  }
  if (std::isnan(rho_mean)) {
    const int64_t np = partial_sum(n_cells, rho, partials.as<double>(), stream);
    reduce_final(partials.as<double>(), np, 1.0 / (double)n_cells, sc, 0, stream);
  } else {
    MG_REQUIRE(std::isfinite(rho_mean), "rho_mean must be finite or NAN");
    MG_HIP(hipStreamSynchronize(stream));   // hp may still be the source of an earlier copy
    hp[4] = rho_mean;
    MG_HIP(hipMemcpyAsync(sc, hp + 4, sizeof(double), hipMemcpyHostToDevice, stream));
  }
  const int64_t n_rhs_partials = u_rhs(n_cells, rho, sc, c, f.as<double>(), partials.as<double>(), stream);
  if (periodic) {
    reduce_final(partials.as<double>(), n_rhs_partials, 1.0, sc, 1, stream);
  } else {
    ghost_values(n_ghost, ghost_idx.as<int32_t>(), phi_parent, ghost_val.as<double>(), stream);
    if (ol[0].n_bricks > 0)
      brick_ghost_pack(ol[0].n_gentries, ol[0].gidx.as<int32_t>(), ghost_val.as<double>(), ol[0].gpack.as<double>(),
                       stream);
    // a refined level's scale is its full right-hand side, f with the
    // Dirichlet terms moved across (the residual of phi = 0)
    const int64_t np = oct_rhs_norm2(n_oct, h, f.as<double>(), ol[0].nbr.as<int32_t>(), ghost_val.as<double>(),
                                     partials.as<double>(), stream);
    reduce_final(partials.as<double>(), np, 1.0, sc, 1, stream);
  }
}

// ||f - L phi||^2 -> scalars[2] (FP64)
void mg_level_s::residual2(const double* phi) {
  double* sc = scalars.as<double>();
  int64_t np = partial_count(n_oct, kReduceBlock);
  if (periodic) {
    np = u_resid_restrict<double>(n, h, phi, f.as<double>(), nullptr, partials.as<double>(), stream);
  } else if (ol[0].n_bricks > 0) {
    brick_resid<double>(ol[0].n_bricks, ol[0].bmap.as<int32_t>(), h, phi, f.as<double>(), nullptr, nullptr,
                        brick_ghosts(true), nullptr, nullptr, nullptr, partials.as<double>(), stream);
    np = ol[0].n_bricks;
  } else {
    oct_resid<double>(n_oct, h, phi, f.as<double>(), ol[0].nbr.as<int32_t>(), nullptr, nullptr,
                      ghost_val.as<double>(), nullptr, nullptr, nullptr, partials.as<double>(), stream);
  }
  reduce_final(partials.as<double>(), np, 1.0, sc, 2, stream);
}

// pre_done (level 0 only): that many pre-smoothing sweeps have already been
// applied by one launch that read e and wrote the level's twin, which now
// holds the current iterate.
template <typename T>
void mg_level_s::vcycle_uniform(int p, int m, T* e0, const T* b0, int pre_done, double* add_into) {
  const int M = (int)un.size() - 1;
  T* e = m == 0 ? e0 : ue[p][m].as<T>();
  const T* b = m == 0 ? b0 : ub[p][m].as<T>();
  const int nm = un[m];
  const double hm = h * (double)(n / nm);
  MG_REQUIRE(add_into == nullptr || (m == 0 && std::is_same<T, float>::value),
             "internal: only an FP32 level-0 cycle adds into an FP64 array");
  auto add_result = [&]() {
    if constexpr (std::is_same<T, float>::value) {
      if (add_into) add_correction((int64_t)nm * nm * nm, add_into, e, stream);
    }
  };
  if (m == M) {
    u_coarse_solve<T>(nm, G[p].as<T>(), b, e, stream);
    add_result();
    return;
  }
  const bool zero_guess = (m > 0) || (p == 1);
  if (zero_guess && small_vcycle(nm) && un[M] == 4) {
    u_vcycle_small<T>(nm, hm, b, e, G[p].as<T>(), desc.nu_pre, desc.nu_post, stream);
    add_result();
    return;
  }
  T* tmp = ut[p][m].as<T>();
  if (tmp != nullptr) {
    // tiled sweeps ping-pong between e and tmp; `cur` holds the current iterate
    T* cur = e;
    T* other = tmp;
    if (pre_done > 0) std::swap(cur, other);   // the head launch wrote tmp
    u_sweeps_tiled<T>(nm, hm, &cur, &other, b, desc.nu_pre - pre_done, zero_guess && pre_done == 0, nullptr, stream);
    u_resid_restrict<T>(nm, hm, cur, b, ub[p][m + 1].as<T>(), nullptr, stream);
    vcycle_uniform<T>(p, m + 1, e0, b0);
    // post-smoothing; its first launch applies the prolongation + correction,
    // its last adds the result to add_into when that is asked for
    const bool fuse_add = add_into != nullptr && desc.nu_post >= 1;
    u_sweeps_tiled<T>(nm, hm, &cur, &other, b, desc.nu_post, false, ue[p][m + 1].as<T>(), stream,
                      fuse_add ? add_into : nullptr);
    if (fuse_add) return;
    if (cur != e) MG_HIP(hipMemcpyAsync(e, cur, (size_t)nm * nm * nm * sizeof(T), hipMemcpyDeviceToDevice, stream));
    add_result();
    return;
  }
  if (zero_guess) u_smooth_zero_guess<T>(nm, hm, e, b, desc.nu_pre, stream, tmp);
  else u_smooth<T>(nm, hm, e, b, desc.nu_pre, stream, tmp);
  u_resid_restrict<T>(nm, hm, e, b, ub[p][m + 1].as<T>(), nullptr, stream);
  vcycle_uniform<T>(p, m + 1, e0, b0);
  u_prolong<T>(nm, ue[p][m + 1].as<T>(), e, stream);
  u_smooth<T>(nm, hm, e, b, desc.nu_post, stream, tmp);
  add_result();
}

template <typename T>
void mg_level_s::vcycle_oct(int p, int m, T* e0, const T* b0, bool ghosts, int pre_done, double* add_into) {
  OctLevel& L = ol[m];
  T* e = m == 0 ? e0 : L.e[p].as<T>();
  MG_REQUIRE(add_into == nullptr || (m == 0 && std::is_same<T, float>::value),
             "internal: only an FP32 level-0 cycle adds into an FP64 array");
  auto add_result = [&]() {
    if constexpr (std::is_same<T, float>::value) {
      if (add_into) add_correction(n_cells, add_into, e, stream);
    }
  };
  const T* b = m == 0 ? b0 : L.b[p].as<T>();
  const uint8_t* mask = L.mask.as<uint8_t>();
  const T* dg = L.diag.as<T>();
  const double* g = (m == 0 && ghosts) ? ghost_val.as<double>() : nullptr;
  if (m == tail_t) {   // this level and all below in one workgroup
    oct_tail<T>(tail_args, tail_blob.p, tail_b.as<T>(), tail_cell.as<int32_t>(), e, stream);
    return;
  }
  // the restriction's target: the next level's b, or the tail's compact one
  const bool into_tail = m + 1 == tail_t;
  const int32_t* fat = into_tail ? tail_father.as<int32_t>() : L.father.as<int32_t>();
  T* bnext = into_tail ? tail_b.as<T>() : ol[m + 1].b[p].as<T>();
  if (m == (int)ol.size() - 1) {
    if (last_smooth_only) {   // pre- and post-smoothing around a zero correction
      const int k = desc.nu_pre + desc.nu_post;
      if (L.n_bricks > 0) {
        T* cur = e;
        T* other = L.t[p].as<T>();
        for (int i = 0; i < k; ++i) {
          brick_sweep<T>(L.n_bricks, L.bmap.as<int32_t>(), L.h, i == 0 ? nullptr : cur, b, other, mask, dg,
                         BrickGhosts{}, stream);
          std::swap(cur, other);
        }
        if (cur != e)
          MG_HIP(hipMemcpyAsync(e, cur, (size_t)L.n_oct * 8 * sizeof(T), hipMemcpyDeviceToDevice, stream));
      } else {
        fill_zero<T>(e, L.n_oct * 8, stream);
        oct_smooth<T>(L.n_oct, L.h, e, b, L.nbr.as<int32_t>(), mask, dg, g, k, stream);
      }
    } else {
      oct_coarsest<T>(L.n_oct, L.h, e, b, L.nbr.as<int32_t>(), mask, dg, coarse_sweeps, stream);
    }
    return;
  }
  const bool zero_guess = m > 0 || p == 1;
  if (L.n_bricks > 0) {
    // fused red+black brick sweeps, ping-pong between e and the twin
    T* cur = e;
    T* other = L.t[p].as<T>();
    if (pre_done > 0) std::swap(cur, other);   // the head launch wrote the twin
    const BrickGhosts gh = brick_ghosts(g != nullptr);
    // ec: the first sweep applies the prolongation of the coarse correction ec;
    // add: the last sweep adds its result to that f64 array (cur is then stale)
    auto sweeps = [&](int k, bool zero_first, const T* ec, double* add = nullptr) {
      for (int i = 0; i < k; ++i) {
        const bool fuse_add = add != nullptr && i == k - 1;
        brick_sweep<T>(L.n_bricks, L.bmap.as<int32_t>(), L.h, (zero_first && i == 0) ? nullptr : cur, b, other, mask,
                       dg, gh, stream, nullptr, L.cmap.as<int32_t>(), L.bshift, i == 0 ? ec : nullptr,
                       fuse_add ? add : nullptr);
        if (!fuse_add) std::swap(cur, other);
      }
      if (k == 0 && zero_first) fill_zero<T>(cur, L.n_oct * 8, stream);
      if (k == 0 && ec)   // no sweep: the prolongation alone
        oct_prolong<T>(L.n_oct, L.father.as<int32_t>(), ol[m + 1].nbr27.as<int32_t>(), ec, cur, mask, stream);
    };
    sweeps(desc.nu_pre - pre_done, zero_guess && pre_done == 0, nullptr);
    brick_resid<T>(L.n_bricks, L.bmap.as<int32_t>(), L.h, cur, b, mask, dg, gh, fat, bnext, nullptr, nullptr,
                   stream);
    vcycle_oct<T>(p, m + 1, e0, b0, ghosts);
    const bool fuse_add = add_into != nullptr && desc.nu_post >= 1;
    sweeps(desc.nu_post, false, ol[m + 1].e[p].as<T>(), fuse_add ? add_into : nullptr);
    if (fuse_add) return;
    if (cur != e) MG_HIP(hipMemcpyAsync(e, cur, (size_t)L.n_oct * 8 * sizeof(T), hipMemcpyDeviceToDevice, stream));
    add_result();
    return;
  }
  if (zero_guess) fill_zero<T>(e, L.n_oct * 8, stream);
  oct_smooth<T>(L.n_oct, L.h, e, b, L.nbr.as<int32_t>(), mask, dg, g, desc.nu_pre, stream);
  oct_resid<T>(L.n_oct, L.h, e, b, L.nbr.as<int32_t>(), mask, dg, g, fat, bnext, nullptr, nullptr, stream);
  vcycle_oct<T>(p, m + 1, e0, b0, ghosts);
  oct_prolong<T>(L.n_oct, L.father.as<int32_t>(), ol[m + 1].nbr27.as<int32_t>(), ol[m + 1].e[p].as<T>(), e, mask,
                 stream);
  oct_smooth<T>(L.n_oct, L.h, e, b, L.nbr.as<int32_t>(), mask, dg, g, desc.nu_post, stream);
  add_result();
}

mg_status_t mg_level_s::solve(const double* rho, double rho_mean, double c, const double* phi_parent, double* phi,
                              double tol, int max_cycles, mg_solve_info_t& info) {
  info = mg_solve_info_t{};
  MG_HIP(hipEventRecord(ev0, stream));
  prepare_rhs(rho, rho_mean, c, phi_parent);
  double* sc = scalars.as<double>();
  float* e32 = nullptr;
  float* r32 = nullptr;
  if (mixed) {
    e32 = periodic ? ue[1][0].as<float>() : ol[0].e[1].as<float>();
    r32 = periodic ? ub[1][0].as<float>() : ol[0].b[1].as<float>();
  }
  // mixed, periodic, n >= 256: the outer residual also takes the correction
  // cycle's first (zero-guess) sweep, writing its result into the level-0 twin
  const bool fused_outer = mixed && periodic && desc.nu_pre >= 1 && fused_outer_resid(n);
  auto outer_residual = [&]() {
    if (!mixed) {
      residual2(phi);
    } else if (fused_outer) {
      const int64_t np =
          u_outer_resid_sweep(n, h, phi, f.as<double>(), r32, ut[1][0].as<float>(), partials.as<double>(), stream);
      reduce_final(partials.as<double>(), np, 1.0, sc, 2, stream);
    } else if (periodic) {
      const int64_t np = u_outer_resid(n, h, phi, f.as<double>(), r32, partials.as<double>(), stream);
      reduce_final(partials.as<double>(), np, 1.0, sc, 2, stream);
    } else if (ol[0].n_bricks > 0) {
      brick_resid<double>(ol[0].n_bricks, ol[0].bmap.as<int32_t>(), h, phi, f.as<double>(), nullptr, nullptr,
                          brick_ghosts(true), nullptr, nullptr, r32, partials.as<double>(), stream);
      reduce_final(partials.as<double>(), ol[0].n_bricks, 1.0, sc, 2, stream);
    } else {
      oct_resid<double>(n_oct, h, phi, f.as<double>(), ol[0].nbr.as<int32_t>(), nullptr, nullptr,
                        ghost_val.as<double>(), nullptr, nullptr, r32, partials.as<double>(), stream);
      reduce_final(partials.as<double>(), partial_count(n_oct, kReduceBlock), 1.0, sc, 2, stream);
    }
  };
  // Plain FP64 solve with tiled (periodic) or brick (refined) sweeps: the
  // first pre-smoothing sweep of each cycle also returns ||f - L phi||^2 of
  // phi as it enters the cycle (it reads phi and writes the twin, so phi is
  // untouched until the check passes); otherwise a separate residual pass
  // follows every cycle.
  const bool fused_norm = !mixed && desc.nu_pre >= 1 && (periodic ? tiled_smoother(n) : ol[0].n_bricks > 0);
  auto head_sweep = [&]() {
    int64_t np = 0;
    if (periodic) {
      np = u_sweep_tiled<double>(n, h, phi, f.as<double>(), ut[0][0].as<double>(), partials.as<double>(), stream);
    } else {
      brick_sweep<double>(ol[0].n_bricks, ol[0].bmap.as<int32_t>(), h, phi, f.as<double>(), ol[0].t[0].as<double>(),
                          nullptr, nullptr, brick_ghosts(true), stream, partials.as<double>());
      np = ol[0].n_bricks;
    }
    reduce_final(partials.as<double>(), np, 1.0, sc, 2, stream);
  };
  if (fused_norm) head_sweep();
  else outer_residual();
  read_scalars(3);
  info.rho_mean = hp[0];
  const double f2 = hp[1];
  if (!(std::isfinite(f2) && std::isfinite(hp[2]))) {
    set_error("mg_solve: non-finite right-hand side or initial residual");
    return MG_ERR_DIVERGED;
  }
  if (f2 == 0.0) {
    // zero right-hand side (periodic: f = 0; refined: f and the Dirichlet
    // terms both zero): the solution is phi = 0
    fill_zero<double>(phi, n_cells, stream);
    MG_HIP(hipStreamSynchronize(stream));
    info.relres = info.relres0 = 0.0;
    return MG_OK;
  }
  const double fn = std::sqrt(f2);
  double relres = std::sqrt(hp[2]) / fn;
  info.relres0 = relres;
  // One unit of work = the rest of a cycle (everything after its head launch)
  // followed by the next cycle's head launch, whose norm is copied into host
  // slot 5 + (unit & 1).  The head launch leaves phi untouched (it writes the
  // twin, or only r32 in mixed precision), so a cycle whose incoming norm is
  // already below tol is never applied.  While the host waits for one unit's
  // norm it enqueues the next unit too, but only when the contraction seen so
  // far says that norm will still be above tol: the GPU then never idles on
  // the host's round trip.  A wrong guess costs one extra cycle, which is kept
  // (phi is then one cycle further converged and its own norm is returned).
  auto unit = [&](int u) {
    if (!mixed) {
      if (periodic) vcycle_uniform<double>(0, 0, phi, f.as<double>(), fused_norm ? 1 : 0);
      else vcycle_oct<double>(0, 0, phi, f.as<double>(), true, fused_norm ? 1 : 0);
    } else {
      if (periodic) {
        vcycle_uniform<float>(1, 0, e32, r32, fused_outer ? 1 : 0, phi);   // adds the correction to phi itself
      } else {
        vcycle_oct<float>(1, 0, e32, r32, false, 0, phi);   // adds the correction to phi itself
      }
    }
    if (fused_norm) head_sweep();
    else outer_residual();
    MG_HIP(hipMemcpyAsync(hp + 5 + (u & 1), sc + 2, sizeof(double), hipMemcpyDeviceToHost, stream));
    MG_HIP(hipEventRecord(evq[u & 1], stream));
  };
  int cycles = 0, queued = 0;
  double prev = 0.0;   // relres one cycle earlier (0: not known yet)
  auto take = [&]() {
    MG_HIP(hipEventSynchronize(evq[cycles & 1]));
    prev = relres;
    relres = std::sqrt(hp[5 + (cycles & 1)]) / fn;
    ++cycles;
  };
  while (relres > tol && cycles < max_cycles) {
    if (queued == cycles) unit(queued++);
    // the norm after the queued unit, predicted from the last contraction
    // (before there is one, a contraction of 1e-3 is assumed)
    const double rate = prev > 0.0 ? std::min(1.0, relres / prev) : 1e-3;
    if (queued == cycles + 1 && queued < max_cycles && relres * rate > 8.0 * tol) unit(queued++);
    take();
    if (!std::isfinite(relres)) {
      MG_HIP(hipStreamSynchronize(stream));
      info.cycles = cycles;
      info.relres = relres;
      set_error("mg_solve: residual norm became non-finite");
      return MG_ERR_DIVERGED;
    }
  }
  if (queued > cycles) {   // a speculative cycle has already been applied to phi
    take();
    if (!std::isfinite(relres)) {
      info.cycles = cycles;
      info.relres = relres;
      set_error("mg_solve: residual norm became non-finite");
      return MG_ERR_DIVERGED;
    }
  }
  if (periodic) {
    const int64_t np = partial_sum(n_cells, phi, partials.as<double>(), stream);
    reduce_final(partials.as<double>(), np, 1.0 / (double)n_cells, sc, 3, stream);
    sub_mean(n_cells, phi, sc + 3, stream);
  }
  MG_HIP(hipEventRecord(ev1, stream));
  MG_HIP(hipEventSynchronize(ev1));
  float ms = 0.f;
  MG_HIP(hipEventElapsedTime(&ms, ev0, ev1));
  info.ms = ms;
  info.cycles = cycles;
  info.relres = relres;
  if (relres > tol) {
    set_error("mg_solve: max_cycles reached before the tolerance");
    return MG_NOT_CONVERGED;
  }
  return MG_OK;
}

mg_status_t mg_level_s::fft_solve(const double* rho, double rho_mean, double c, double* phi,
                                  mg_solve_info_t& info) {
  info = mg_solve_info_t{};
  MG_REQUIRE(periodic, "mg_fft_solve: only a periodic (level 0) handle has a direct FFT solve");
  MG_REQUIRE(n >= 8 && n <= fft_max_n(), "mg_fft_solve: n must be in [8, " + std::to_string(fft_max_n()) + "]");
  if (fft_work.p == nullptr) {
    fft_tables(n, h, fft_tw, fft_lam, stream);
    fft_work.alloc(fft_work_bytes(n));
    // partial sums: one per x-pass workgroup (the mean), two per residual tile
    const int64_t need =
        std::max<int64_t>((int64_t)(n / 2) * (n / 2), tiled_smoother(n) ? 2 * tiled_sweep_blocks(n) : 0);
    if (need > n_partials) {
      MG_HIP(hipStreamSynchronize(stream));
      n_partials = need;
      partials.alloc(n_partials * sizeof(double));
    }
  }
  MG_REQUIRE(std::isnan(rho_mean) || std::isfinite(rho_mean), "mg_fft_solve: rho_mean must be finite or NAN");
  double* sc = scalars.as<double>();
  if (!std::isnan(rho_mean)) {
    MG_HIP(hipStreamSynchronize(stream));   // hp may still be the source of an earlier copy
    hp[4] = rho_mean;
  }
  MG_HIP(hipEventRecord(ev0, stream));
  if (tiled_smoother(n)) {
    // the transforms read rho itself (the mean only moves the zero mode, which
    // the solve sets to 0) and sum it for the mean; the residual check forms f
    // on the fly: f is never stored
    const bool want_mean = std::isnan(rho_mean);
    if (!want_mean) MG_HIP(hipMemcpyAsync(sc, hp + 4, sizeof(double), hipMemcpyHostToDevice, stream));
    mg::fft_solve(n, rho, c, phi, fft_work.p, fft_tw.p, fft_lam.as<double>(),
                  want_mean ? partials.as<double>() : nullptr, stream);
    if (want_mean)
      reduce_final(partials.as<double>(), (int64_t)(n / 2) * (n / 2), 1.0 / (double)n_cells, sc, 0, stream);
    double* pr = partials.as<double>();
    double* pf = pr + tiled_sweep_blocks(n);
    const int64_t np = u_resid_from_rho(n, h, phi, rho, c, sc, pr, pf, stream);
    reduce_final(pr, np, 1.0, sc, 2, stream);
    reduce_final(pf, np, 1.0, sc, 1, stream);
  } else {
    prepare_rhs(rho, rho_mean, c, nullptr);
    mg::fft_solve(n, f.as<double>(), 1.0, phi, fft_work.p, fft_tw.p, fft_lam.as<double>(), nullptr, stream);
    residual2(phi);
  }
  MG_HIP(hipEventRecord(ev1, stream));
  read_scalars(3);
  float ms = 0.f;
  MG_HIP(hipEventElapsedTime(&ms, ev0, ev1));
  info.ms = ms;
  info.rho_mean = hp[0];
  const double f2 = hp[1];
  if (!(std::isfinite(f2) && std::isfinite(hp[2]))) {
    set_error("mg_fft_solve: non-finite right-hand side or residual");
    return MG_ERR_DIVERGED;
  }
  if (f2 == 0.0) {   // f = 0: phi = 0 exactly (the transforms of a constant density leave rounding noise)
    fill_zero<double>(phi, n_cells, stream);
    MG_HIP(hipStreamSynchronize(stream));
    info.relres = info.relres0 = 0.0;
    return MG_OK;
  }
  info.relres0 = 1.0;   // the zero guess
  info.relres = std::sqrt(hp[2] / f2);
  return MG_OK;
}

void mg_level_s::residual_norm(const double* rho, double rho_mean, double c, const double* phi_parent,
                               const double* phi, double& rn, double& fn) {
  prepare_rhs(rho, rho_mean, c, phi_parent);
  residual2(phi);
  read_scalars(3);
  rn = std::sqrt(hp[2]);
  fn = std::sqrt(hp[1]);
}

void mg_level_s::smooth(const double* rho, double rho_mean, double c, const double* phi_parent, double* phi,
                        int sweeps) {
  prepare_rhs(rho, rho_mean, c, phi_parent);
  if (periodic) {
    u_smooth<double>(n, h, phi, f.as<double>(), sweeps, stream, tiled_smoother(n) ? ut[0][0].as<double>() : nullptr);
  } else {
    OctLevel& L = ol[0];
    if (L.n_bricks > 0) {
      double* cur = phi;
      double* other = L.t[0].as<double>();
      const BrickGhosts gh = brick_ghosts(true);
      for (int i = 0; i < sweeps; ++i) {
        brick_sweep<double>(L.n_bricks, L.bmap.as<int32_t>(), L.h, cur, f.as<double>(), other, nullptr, nullptr, gh,
                            stream);
        std::swap(cur, other);
      }
      if (cur != phi) MG_HIP(hipMemcpyAsync(phi, cur, (size_t)n_oct * 8 * sizeof(double), hipMemcpyDeviceToDevice, stream));
    } else {
      oct_smooth<double>(n_oct, h, phi, f.as<double>(), L.nbr.as<int32_t>(), nullptr, nullptr, ghost_val.as<double>(),
                         sweeps, stream);
    }
  }
  MG_HIP(hipStreamSynchronize(stream));
}

void mg_level_s::force(const double* phi_parent, const double* phi, double* g) {
  if (periodic) {
    MG_REQUIRE(phi_parent == nullptr, "mg_force: periodic level: d_phi_parent must be NULL");
    u_force(n, h, phi, g, stream);
  } else {
    MG_REQUIRE(phi_parent != nullptr, "mg_force: refined level: d_phi_parent is required");
    ghost_values(n_ghost, ghost_idx.as<int32_t>(), phi_parent, ghost_val.as<double>(), stream);
    oct_force(n_oct, h, phi, ol[0].nbr.as<int32_t>(), ghost_val.as<double>(), g, stream);
  }
  MG_HIP(hipStreamSynchronize(stream));
}

void mg_level_s::get_neighbors(int32_t* d_nbr) {
  MG_REQUIRE(!periodic, "mg_get_neighbors: a periodic level has no neighbour cache (neighbours are implicit)");
  nbr_export(n_oct, ol[0].nbr.as<int32_t>(), d_nbr, stream);
  MG_HIP(hipStreamSynchronize(stream));
}

std::vector<int64_t> mg_level_s::active_cells() const {
  std::vector<int64_t> a;
  if (periodic) {
    for (int m : un) a.push_back((int64_t)m * m * m);
  } else {
    for (const OctLevel& L : ol) a.push_back(L.n_active);
  }
  return a;
}

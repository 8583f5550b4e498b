// The level handle: multigrid hierarchy and solve drivers.
#pragma once

#include "mg_internal.h"

namespace mg {

// One multigrid level built from a list of octs (a refined level, or a coarse
// level of its father-cell hierarchy).  nbr[o][j] >= 0 is a neighbour oct;
// -1 is an absent neighbour (value 0 in the error equation); <= -2 encodes
// the ghost face g = -2 - nbr (finest level only, 4 ghost values per face).
struct OctLevel {
  int64_t n_oct = 0;
  int n_dim = 0;            // octs per dimension of the level's full extent
  double h = 0.0;
  DevBuf keys;              // u64 Morton keys of the oct coordinates
  DevBuf nbr;               // i32 [n_oct][6]
  DevBuf mask;              // u8 [n_oct] active-cell bits (coarse levels), NULL = all active
  DevBuf lsm;               // f32 [n_oct][8] level-set mask (coarse levels)
  DevBuf father;            // i32 [n_oct] flat coarse cell index on the next level
  DevBuf nbr27;             // i32 [n_oct][27] octs at offsets (dx,dy,dz) in {-1,0,1}^3 (coarse levels)
  DevBuf diag;              // [n_oct][8] diagonal of the coarse error operator, precision of the cycle
  int64_t n_active = 0;
  // per-precision work arrays (index 0: f64, 1: f32); level 0 of the f64
  // hierarchy uses the caller's phi and the handle's f
  DevBuf e[2], b[2];
  // brick sweeps (levels spanning >= 4 octs per dimension, except the coarsest)
  int64_t n_bricks = 0;
  int bshift = 0;           // brick lattice shift (bit a: one oct along axis a)
  DevBuf bmap;              // i32 [n_bricks][216] oct box maps
  DevBuf cmap;              // i32 [n_bricks][125] coarse octs of each brick's coarse box (next level)
  DevBuf t[2];              // ping-pong twin of e (level 0, f64: of the caller's phi)
  DevBuf gfirst, gcell, gidx;   // per-brick ghost lists (level 0 of a refined level)
  DevBuf gpack;                 // f64 value of each list entry, gathered per solve
  int64_t n_gentries = 0;
};

struct HashTable {
  DevBuf slots;             // {u64 key, i32 value, i32 pad} x capacity
  int64_t capacity = 0;
};

}  // namespace mg

struct mg_level_s {
  mg_level_desc_t desc{};
  hipStream_t stream = nullptr;
  bool periodic = true;
  int64_t n_oct = 0, n_cells = 0;
  int n = 0;                 // cells per dimension of the level's full extent
  double h = 0.0;
  bool mixed = false;
  int coarsest_n = 4;

  // --- periodic level: uniform hierarchy n, n/2, ..., 4 ---
  std::vector<int> un;                      // cells per dimension per level
  std::vector<mg::DevBuf> ue[2], ub[2];     // [prec][m] (m >= 1 for f64; m >= 0 for f32)
  std::vector<mg::DevBuf> ut[2];            // [prec][m] ping-pong twin of the level's phi/e (tiled sweeps)
  mg::DevBuf G[2];                          // coarsest pseudo-inverse per precision

  // --- refined level ---
  // Key frame.  Oct keys are 64-bit Morton keys (21 bits per axis) of the oct
  // coordinates relative to `frame` (octs, per axis), in a key space of
  // `key_dim` octs per dimension.  A level whose extent fits 21 bits keeps
  // frame 0 and key_dim = its extent (periodic wrap at the extent); a deeper
  // level takes key_dim = 2^21 and a frame a little below its octs' bounding
  // box, so no neighbour step wraps inside the key space.
  int64_t frame[3] = {0, 0, 0};
  int64_t key_dim = 0;
  mg::DevArena arena;                       // the refined level's device buffers
  mg::HashTable hash;
  std::vector<mg::OctLevel> ol;            // ol[0] = this level's octs
  mg::DevBuf ghost_idx;                     // i32 [n_ghost][4][8] parent flat cell indices
  mg::DevBuf ghost_val;                     // f64 [n_ghost][4]
  int64_t n_ghost = 0;
  int coarse_sweeps = 64;
  bool last_smooth_only = false;            // the hierarchy ends above a level without active cells
  // levels tail_t .. last cycled in one workgroup (-1: none), tables in the
  // cycle's precision (see mg::oct_tail); tail_b: the first tail level's
  // compact right-hand side, written through tail_father (per oct of level
  // tail_t - 1: the compact index of its father cell, -1 if inactive)
  int tail_t = -1;
  mg::TailArgs tail_args;
  mg::DevBuf tail_blob, tail_b, tail_father, tail_cell;

  // --- direct FFT solve (periodic level; allocated at its first use) ---
  mg::DevBuf fft_work, fft_tw, fft_lam;

  // --- shared scratch ---
  mg::DevBuf f;                             // f64 right-hand side of this level
  mg::DevBuf partials;
  int64_t n_partials = 0;
  mg::DevBuf scalars;                       // f64 [8] on device
  double* hp = nullptr;                     // pinned host mirror of scalars
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evq[2] = {nullptr, nullptr};   // per-unit norm copies of the pipelined solve

  ~mg_level_s();
  void build(const mg_level_desc_t& d);
  mg_status_t solve(const double* rho, double rho_mean, double c, const double* phi_parent, double* phi,
                    double tol, int max_cycles, mg_solve_info_t& info);
  void residual_norm(const double* rho, double rho_mean, double c, const double* phi_parent,
                     const double* phi, double& rn, double& fn);
  void smooth(const double* rho, double rho_mean, double c, const double* phi_parent, double* phi, int sweeps);
  mg_status_t fft_solve(const double* rho, double rho_mean, double c, double* phi, mg_solve_info_t& info);
  void force(const double* phi_parent, const double* phi, double* g);
  void get_neighbors(int32_t* d_nbr);
  std::vector<int64_t> active_cells() const;

  // parent-cell lookup support for a child level's ghosts
  bool is_uniform() const { return periodic; }

 private:
  void build_uniform();
  void build_refined();
  template <typename T>
  void build_tail(int t);
  void prepare_rhs(const double* rho, double rho_mean, double c, const double* phi_parent);
  void residual2(const double* phi);   // ||f - L phi||^2 into scalars[2] (async) + host read
  // add_into (level 0): the cycle's result e0 is added to this f64 array
  // (e0 itself is then left undefined)
  template <typename T>
  void vcycle_uniform(int p, int m, T* e0, const T* b0, int pre_done = 0, double* add_into = nullptr);
  // pre_done, add_into (level 0): as for vcycle_uniform
  template <typename T>
  void vcycle_oct(int p, int m, T* e0, const T* b0, bool ghosts, int pre_done = 0, double* add_into = nullptr);
  mg::BrickGhosts brick_ghosts(bool with_values) const;
  void read_scalars(int count);
};

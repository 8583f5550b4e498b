/*
 * mg.h -- C ABI of the MI355X (gfx950) multigrid Poisson solver for one level
 * of an oct-based adaptive mesh.
 *
 * Problem (section "Poisson solver optimizations", subsection "Multi-Grid
 * Method"; equation gs_update and the fused residual of the appendix
 * "Multigrid solver implementation details"):
 *
 *     L_h phi = f,   f = four_pi_G * (rho - rho_mean),
 *     (L_h phi)_c = (sum of the 6 face neighbours of c - 6 phi_c) / h^2,
 *
 * on the unit box, h = 1 / (base_n * 2^level).  Level 0 is periodic and
 * fully populated; phi is returned with mean 0.  A refined level (level >= 1)
 * holds an arbitrary set of octs; a face neighbour whose oct is absent is a
 * ghost, set to the trilinear interpolation of the parent level's phi
 * (Dirichlet boundary; the interpolation stencil reads neighbouring coarse
 * cells as in the V-cycle subsection).  The solver runs multigrid V-cycles
 * (red-black Gauss-Seidel smoothing, fused residual + restriction by the mean
 * of 8 children, trilinear prolongation + correction, direct coarsest solve;
 * algorithm "GPU-accelerated V-cycle") until ||f - L_h phi||_2 / ||b||_2 <= tol,
 * b the right-hand side of the level's linear system (see mg_solve).
 *
 * Memory layout of every field argument ("oct-major"): [n_oct][8] values,
 * cell c = cx + 2*cy + 4*cz inside an oct (an oct is a 2x2x2 block of cells,
 * the paper's "grid").  On a full periodic level octs are lexicographic with
 * x fastest: oct = (oz * no + oy) * no + ox, no = n / 2.  On a refined level
 * octs are in the order of the d_oct_ijk array given at build time.
 *
 * Conventions
 *  - Pointers named d_* are DEVICE pointers owned by the caller; the library
 *    never frees them or keeps them past the call.  h_* are host pointers.
 *    Field arrays (d_rho, d_phi, d_phi_parent and the d_* arrays of the mg_op_*
 *    calls) must be 16-byte aligned, as every hipMalloc / torch allocation is;
 *    a misaligned pointer is rejected with MG_ERR_ARG.
 *  - The handle owns every internal allocation (hash table, neighbour cache,
 *    multigrid hierarchy, scratch).  A handle is not thread-safe: use one
 *    handle per host thread / stream.
 *  - All device work is enqueued on the stream given at build time (NULL =
 *    the default stream).  mg_solve synchronises that stream once per V-cycle
 *    to read the 8-byte residual norm; mg_residual_norm returns synchronously.
 *  - Every call validates its arguments on the host before launching any
 *    kernel and returns a status; no call aborts or exits.  On a non-OK
 *    status mg_last_error() holds a message (per host thread).
 */
#ifndef MG_H_
#define MG_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_level_s* mg_level_t;

typedef enum {
  MG_OK = 0,
  MG_NOT_CONVERGED = 1,   /* warning: max_cycles reached; d_phi holds the last iterate */
  MG_ERR_ARG = -1,        /* invalid argument (null pointer, bad size, duplicate oct, ...) */
  MG_ERR_OOM = -2,        /* device allocation failed */
  MG_ERR_HIP = -3,        /* HIP runtime error (message in mg_last_error) */
  MG_ERR_TABLE = -4,      /* hash table cannot hold the octs at the requested load factor */
  MG_ERR_DIVERGED = -5,   /* residual norm became NaN or Inf */
  MG_ERR_NESTING = -6     /* a ghost's coarse interpolation stencil is missing on the parent */
} mg_status_t;

enum { MG_PREC_FP64 = 0, MG_PREC_MIXED = 1 };

typedef struct {
  int32_t base_n;            /* level-0 cells per dimension: power of two, 8 <= base_n <= 4096 */
  int32_t level;             /* 0 = periodic base level; >= 1 = refined level; at most 30 and
                                base_n * 2^(level-1) <= 2^31 (oct coordinates are int32) */
  int64_t n_oct;             /* octs on this level; level 0 requires (base_n/2)^3 */
  const int32_t* d_oct_ijk;  /* level >= 1: [n_oct][3] oct coordinates, each in
                                [0, base_n * 2^level / 2), all distinct.  Must be NULL on level 0.
                                A level wider than 2^21 octs per axis is keyed relative to a
                                frame near its octs, which must then lie within 2^21 - 4
                                consecutive octs (periodically) along each axis. */
  mg_level_t parent;         /* level >= 1: handle of level-1 (source of the Dirichlet ghosts) */
  int32_t nu_pre;            /* red-black sweeps before restriction (paper: n_gs; default 2) */
  int32_t nu_post;           /* red-black sweeps after prolongation (default 2) */
  int32_t coarsest_n;        /* level 0: cells per dimension of the coarsest grid of the
                                hierarchy base_n, base_n/2, ..., coarsest_n, where the coarse
                                error equation is solved exactly (the paper's direct coarsest
                                solve; its pseudo-inverse, the system being singular on a
                                periodic grid): 2, 4 or 8, at most base_n; 0 selects 4.
                                Refined levels accept the same values and ignore them: their
                                father-cell hierarchy ends at the first level small enough for
                                one workgroup, which red-black sweeps relax. */
  int32_t brick_shift;       /* refined levels: lattice of the 4x4x4-oct bricks in which the sweeps
                                stage octs in LDS.  0 (default) picks, per hierarchy level, the
                                one of the 8 lattices shifted by 0 or 1 oct along each axis that
                                covers the octs with the fewest bricks; 1 + sx + 2 sy + 4 sz forces
                                the shift (sx, sy, sz) on every level.  Results do not depend on it
                                beyond the order in which the residual norm is summed.  Periodic
                                levels ignore it.  Must be in [0, 8]. */
  int32_t precision;         /* MG_PREC_FP64, or MG_PREC_MIXED (FP32 V-cycles in an FP64
                                defect-correction loop) */
  double load_factor;        /* hash-table load factor in (0, 0.9]; capacity = smallest power
                                of two >= n_oct / load_factor (default 0.5) */
  void* stream;              /* hipStream_t for all work of this handle (NULL = default) */
} mg_level_desc_t;

typedef struct {
  int32_t cycles;            /* V-cycles (plain) or outer corrections (mixed) performed */
  double relres;             /* final relative residual ||f - L phi|| / ||b|| (FP64; b as in mg_solve) */
  double relres0;            /* same for the initial guess */
  double rho_mean;           /* the mean used in f */
  double ms;                 /* wall time of the solve on the stream (hipEvent) */
  int32_t used_fallback;     /* mgnn_solve_warm: 1 when the network's guess was rejected and the
                                solve started from zero; 0 otherwise (always 0 from mg_solve) */
} mg_solve_info_t;

/* Build a level: validates the description, then (on the GPU, on desc->stream)
 * builds the Morton-key hash table of the octs (level >= 1; section "Morton
 * key encoding and neighbour arithmetic", equation hash_func), the neighbour
 * cache (equation nbor_precompute), the Dirichlet ghost stencils against the
 * parent level, and the multigrid hierarchy.  Keys are 64-bit Morton keys of
 * the oct coordinates; on levels wider than 21 bits per axis (where the
 * paper switches to 128-bit keys) they are taken relative to a per-level
 * frame, which keeps 64-bit keys, table slots and compare-and-swap.  The
 * parent handle must outlive this one.  *out receives the handle; on failure
 * *out is NULL. */
mg_status_t mg_build_level(const mg_level_desc_t* desc, mg_level_t* out);

/* Solve L_h phi = four_pi_G (rho - rho_mean) on the level.
 *  d_rho        [n_oct][8] f64 density (read only).
 *  rho_mean     mean density; pass NAN on a periodic level to use the FP64
 *               mean of d_rho (computed on the GPU).  Required (finite) on
 *               refined levels: it is the base level's mean.
 *  d_phi_parent parent level's phi in the parent's layout (refined levels);
 *               must be NULL on level 0.
 *  d_phi        [n_oct][8] f64, in/out: initial guess in (zeros or a warm
 *               start), solution out.  Periodic levels: mean 0 on return.
 *  tol          stop when ||f - L phi||_2 / ||b||_2 <= tol (FP64 residual), where b is
 *               the right-hand side of the level's linear system: b = f on a periodic
 *               level; on a refined level b = f - (sum of each cell's ghost
 *               neighbours) / h^2, the Dirichlet terms moved across (the residual of
 *               phi = 0, so a zero guess has relative residual 1, and a level driven
 *               only by its boundary is measured on that boundary's scale).  The
 *               test uses the library's own FP64 residual; an independent FP64
 *               evaluation of the same phi differs by rounding of relative size
 *               ~ 1e-16 * ||L|| ||phi|| / ||b||, which grows as 1/h^2 and can reach
 *               1e-11 on levels finer than 2^22 cells per axis: ask for a tolerance
 *               below the one that must hold there.
 *  max_cycles   upper bound on V-cycles (outer corrections in mixed mode).
 *  info         optional (may be NULL).
 * A zero right-hand side (b = 0) returns phi = 0 at once.
 * Returns MG_OK, MG_NOT_CONVERGED (d_phi holds the last iterate), or an error. */
mg_status_t mg_solve(mg_level_t L, const double* d_rho, double rho_mean, double four_pi_G,
                     const double* d_phi_parent, double* d_phi, double tol,
                     int32_t max_cycles, mg_solve_info_t* info);

/* n_sweeps red-black Gauss-Seidel sweeps (equation gs_update, red cells
 * first) of the level's own equation L_h phi = four_pi_G (rho - rho_mean),
 * in FP64, applied in place to d_phi [n_oct][8]: the smoother of the V-cycle
 * on its finest level.  Refined levels take their Dirichlet ghosts from
 * d_phi_parent; rho_mean as in mg_solve.  n_sweeps >= 0.  Synchronous. */
mg_status_t mg_level_smooth(mg_level_t L, const double* d_rho, double rho_mean, double four_pi_G,
                            const double* d_phi_parent, double* d_phi, int32_t n_sweeps);

/* FP64 residual norms of a given phi (the fused residual + norm of the MG
 * appendix): *res_norm = ||f - L_h phi||_2 and *rhs_norm = ||b||_2 (b as in
 * mg_solve: f on periodic levels, f minus the ghost terms on refined ones),
 * with ghosts from d_phi_parent on refined levels and rho_mean as in mg_solve
 * (NAN allowed on periodic levels).  Synchronous; host outputs. */
mg_status_t mg_residual_norm(mg_level_t L, const double* d_rho, double rho_mean,
                             double four_pi_G, const double* d_phi_parent,
                             const double* d_phi, double* res_norm, double* rhs_norm);

/* Direct solve of a periodic level (level 0 handle, n^3 cells with n in
 * [8, 1024]) by FFT, as the paper's base-level solver does (section "FFTW3
 * CPU Direct Poisson Solver": forward FFT, Green's function multiply, inverse
 * FFT), with the Green's function of the discrete 7-point operator: d_phi
 * receives the exact solution of the system mg_solve iterates on, with mean 0
 * (up to rounding; info->relres is its FP64 relative residual, typically
 * ~1e-14).  d_rho, rho_mean, four_pi_G as in mg_solve; d_phi is output only
 * ([n_oct][8] f64).  The first call on a handle allocates about n^3 / 2
 * complex doubles of work space, kept until mg_destroy_level.  info (optional) gets cycles =
 * 0, relres0 = 1 (the zero guess), relres, rho_mean and ms.  Synchronous.
 * Returns MG_OK, MG_ERR_ARG (refined level, n out of range) or an error. */
mg_status_t mg_fft_solve(mg_level_t L, const double* d_rho, double rho_mean, double four_pi_G,
                         double* d_phi, mg_solve_info_t* info);

/* Solve a whole hierarchy coarse to fine, as the paper's gravity step walks
 * the AMR levels (section "Multi-Grid Method": each refined level takes its
 * Dirichlet boundary values from the level above): level 0 by V-cycles, or
 * by the direct FFT solve when base_fft != 0, then every refined level i by
 * mg_solve with the potential of level i-1 as its parent.
 *  levels[i]   built as level i, with parent levels[i-1] (i >= 1)
 *  d_rho[i], d_phi[i]  the level's density and potential (as in mg_solve;
 *              d_phi[i] holds the initial guess on entry for i >= 1, and for
 *              i = 0 unless base_fft)
 *  rho_mean    NAN: the FP64 mean of level 0's density, used on every level
 *  infos       optional, n_levels entries
 * Synchronous.  A level that reaches max_cycles (MG_NOT_CONVERGED) does not
 * stop the chain; an error does (the levels after it are left untouched).
 * Returns MG_OK, MG_NOT_CONVERGED if any level did not converge, or the
 * first error. */
mg_status_t mg_solve_chain(const mg_level_t* levels, int32_t n_levels, const double* const* d_rho,
                           double rho_mean, double four_pi_G, double* const* d_phi, double tol,
                           int32_t max_cycles, int32_t base_fft, mg_solve_info_t* infos);

/* Gravitational acceleration g = -grad(phi) of a level's potential, the
 * per-cell force step that follows the solve (section "GPU offloading:
 * approach and assessment" lists it; the paper prints no stencil): second-
 * order central differences g_d = (phi(c - e_d) - phi(c + e_d)) / (2h), the
 * gradient that matches the 7-point operator.  Periodic levels wrap; on a
 * refined level a neighbour outside the level's octs is its ghost, the
 * trilinear interpolation of d_phi_parent the solve uses.
 *  d_phi_parent parent level's phi (refined levels); NULL on level 0.
 *  d_phi        [n_oct][8] f64 (read only).
 *  d_force      [3][n_oct][8] f64 output, component-major (x, y, z), same
 *               oct order as d_phi; must not overlap d_phi.
 * Synchronous.  Returns MG_OK or MG_ERR_ARG (NULL or misaligned arrays, a
 * parent potential on level 0 or none on a refined level). */
mg_status_t mg_force(mg_level_t L, const double* d_phi_parent, const double* d_phi, double* d_force);

/* Copy the level's neighbour cache to d_nbr [n_oct][6] int32 (directions -x,
 * +x, -y, +y, -z, +z): the index of the same-level neighbour oct, or -1 when
 * absent (periodic wrap at the level's extent).  Test hook for the hash table. */
mg_status_t mg_get_neighbors(mg_level_t L, int32_t* d_nbr);

/* Number of levels in the handle's multigrid hierarchy and active cells on
 * level m (h_active_cells must hold n_levels entries).  On refined levels the
 * hierarchy ends above the first father-cell level without active cells (its
 * correction would be zero). */
mg_status_t mg_hierarchy_info(mg_level_t L, int32_t* n_levels, int64_t* h_active_cells,
                              int32_t capacity);

void mg_destroy_level(mg_level_t L);

/* Message for the last non-OK status returned on this host thread. */
const char* mg_last_error(void);

/* ------------------------------------------------------------------------
 * Kernel-level entry points on a full periodic grid (n^3 cells, oct-major,
 * n a power of two >= 4), used for step-by-step parity checks.  dtype: 0 =
 * f64, 1 = f32 (all array arguments of the call have that type).  Work is
 * enqueued on `stream`; the calls do not synchronise.
 * ------------------------------------------------------------------------ */

/* n_sweeps red-black Gauss-Seidel sweeps in place on d_phi (equation
 * gs_update): each sweep updates every red cell ((i+j+k) even), then every
 * black cell, with phi_c <- (sum of 6 neighbours - h^2 b_c) * (1/6).
 * d_work: optional device scratch of n^3 elements of dtype (the fused tiled
 * sweep reads one buffer and writes the other); NULL = the library allocates
 * it for the call (and synchronises the stream before freeing it). */
mg_status_t mg_op_smooth(int32_t n, double h, int32_t dtype, void* d_phi, const void* d_b,
                         int32_t n_sweeps, void* d_work, void* stream);

/* Fused residual + restriction + norm: r = b - L_h phi on the n^3 grid;
 * d_bc[(n/2)^3] (oct-major at n/2) = mean of each cell's 8 children;
 * *d_norm2 (f64, device) = sum of r^2 accumulated in f64.  d_norm2 may be NULL. */
mg_status_t mg_op_resid_restrict(int32_t n, double h, int32_t dtype, const void* d_phi,
                                 const void* d_b, void* d_bc, double* d_norm2, void* stream);

/* mg_op_resid_restrict for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the per-workgroup norm
 * partials in a static device array of the library (4 MiB per GPU, held until
 * the process ends) instead of a buffer allocated per call.  n <= 1024 (the
 * partials must fit that array; larger n returns MG_ERR_ARG).  Calls no
 * allocating routine and does not synchronise: the work is enqueued on
 * `stream`.  The array is shared by every call on one GPU, so calls that
 * overlap on one GPU (concurrent streams or host threads) race on it; calls
 * ordered on one stream do not.  Nothing in it needs to start at zero (every
 * partial is written before it is read). */
mg_status_t mg_op_resid_restrict_noalloc(int32_t n, double h, int32_t dtype, const void* d_phi,
                                         const void* d_b, void* d_bc, double* d_norm2, void* stream);

/* g = -grad(phi) on the periodic n^3 grid (f64 only; mg_force's periodic
 * case): d_force [3][n^3], component-major, oct-major within a component. */
mg_status_t mg_op_force(int32_t n, double h, const double* d_phi, double* d_force, void* stream);

/* Prolongation + correction: d_e[n^3] += trilinear (cell-centred, periodic)
 * interpolation of d_ec[(n/2)^3]. */
mg_status_t mg_op_prolong(int32_t n, int32_t dtype, const void* d_ec, void* d_e, void* stream);

/* Exact coarsest solve on n^3 periodic cells, n in {2, 4, 8}: d_e = A^+ d_b
 * (the mean-free minimum-norm solution). */
mg_status_t mg_op_coarse_solve(int32_t n, double h, int32_t dtype, const void* d_b, void* d_e,
                               void* stream);

/* Morton keys of oct coordinates (equation morton_encode, 21 bits per axis):
 * d_keys[i] = interleave(d_ijk[3i], d_ijk[3i+1], d_ijk[3i+2]). */
mg_status_t mg_op_morton(int64_t n, const int32_t* d_ijk, uint64_t* d_keys, void* stream);

/* Layout helpers for a full periodic field of n^3 f64 values (n a power of
 * two in [2, 4096]): the dense array indexed (x n + y) n + z (z fastest; cell
 * (x, y, z) has centre ((x, y, z) + 1/2) / n) and the oct-major layout of a
 * periodic level (see the top of this file), the order every field argument
 * above uses.  The paper stores cells per grid (oct) in its own arrays; these
 * calls move a caller's dense grid onto that layout and back.  A pure
 * permutation (bit-exact).  d_dense and d_oct are device arrays of n^3 f64,
 * 16-byte aligned, not overlapping.  Asynchronous on `stream`.  Returns
 * MG_OK or MG_ERR_ARG. */
mg_status_t mg_dense_to_oct(int32_t n, const double* d_dense, double* d_oct, void* stream);
mg_status_t mg_oct_to_dense(int32_t n, const double* d_oct, double* d_dense, void* stream);

/* Table hash of n keys (appendix "Per-level hash table and replacement
 * functions", equation hash_func): each key is reduced to 64 bits (key_words
 * = 1: the key itself; 2: XOR of its low and high words, keys laid out as in
 * the key table below), then t = ((h * 2654435761) ^ (h >> 16)) *
 * 0x9E3779B97F4A7C15 and h(M) = t ^ (t >> 13) in unsigned 64-bit arithmetic:
 * d_hash[i] = h(M_i).  A key's home slot in a table of capacity C (a power of
 * two) is h(M) & (C - 1), in the level builder's table and in the key table
 * alike.  Test hook; asynchronous on `stream`.  Returns MG_OK or MG_ERR_ARG
 * (key_words not 1 or 2, NULL or misaligned arrays). */
mg_status_t mg_op_hash(int64_t n, int32_t key_words, const uint64_t* d_keys, uint64_t* d_hash, void* stream);

/* ------------------------------------------------------------------------
 * Incrementally maintained Morton-key table (appendix "Per-level hash table
 * and replacement functions": a grid is inserted when it is made and deleted
 * when it is killed; a rebuild drops deleted entries), for 64-bit keys (B = 21
 * bits per coordinate, levels whose extent is at most 2^21 octs per
 * dimension) or 128-bit keys (B = 42, up to 2^42; section "Morton key
 * encoding and neighbour arithmetic").  The level builder above keeps its own
 * 64-bit table; this one is for callers that add and remove grids between
 * solves, and for levels deeper than 64-bit keys reach.
 *
 * Keys are device arrays of uint64: one word per key (key_words = 1) or two,
 * low word first (key_words = 2), laid out as mg_op_morton / mg_op_morton128
 * write them.  A key must leave bit 63 (64-bit) or bits 62-63 of its high word
 * (128-bit) clear, as every Morton key does; those values mark empty and
 * deleted slots.  Values are int32 grid indices (any value; lookups return -1
 * for an absent key, so -1 is best not stored).  Open addressing with linear
 * probing on the hash of equation hash_func (128-bit keys: of the XOR of the
 * two words); the table doubles automatically so that live plus deleted
 * entries stay at or below max_load of the capacity.  Work is enqueued on the
 * table's stream; insert, erase and rebuild synchronise it (they read back
 * the counts that decide the next rehash), lookup and neighbours do not.
 * Not thread-safe: one table per stream.
 * ------------------------------------------------------------------------ */
typedef struct mg_hash_s* mg_hash_t;

/* New empty table: key_words 1 or 2; capacity: initial slots (rounded up to a
 * power of two, at least 16; 0 = minimal); max_load in (0, 0.9] (the paper
 * keeps 0.7); stream: hipStream_t or NULL for the default stream. */
mg_status_t mg_hash_create(int32_t key_words, int64_t capacity, double max_load, void* stream,
                           mg_hash_t* out);
void mg_hash_destroy(mg_hash_t H);

/* Insert or assign n keys with values d_vals[n] (int32).  A key already in
 * the table takes its new value; a key repeated within one call is stored
 * once, with one of its values.  MG_ERR_ARG if a key has the reserved bits
 * set (such keys are skipped, the others inserted). */
mg_status_t mg_hash_insert(mg_hash_t H, int64_t n, const uint64_t* d_keys, const int32_t* d_vals);

/* Delete n keys (absent keys are ignored; repeats count once). */
mg_status_t mg_hash_erase(mg_hash_t H, int64_t n, const uint64_t* d_keys);

/* d_vals[i] = value of key i, or -1 when absent.  Asynchronous. */
mg_status_t mg_hash_lookup(mg_hash_t H, int64_t n, const uint64_t* d_keys, int32_t* d_vals);

/* Neighbour cache rows (equation nbor_precompute) for n keys of one level
 * with n_dim octs per dimension (a power of two, at most 2^21 or 2^42):
 * d_nbr[n][6] int32 = value of the key one step away in -x, +x, -y, +y, -z,
 * +z (periodic wrap at n_dim), or -1.  Asynchronous. */
mg_status_t mg_hash_neighbours(mg_hash_t H, int64_t n, const uint64_t* d_keys, int64_t n_dim,
                               int32_t* d_nbr);

/* Rebuild without deleted entries at the smallest power-of-two capacity (>= 16)
 * that holds the live entries within max_load. */
mg_status_t mg_hash_rebuild(mg_hash_t H);

/* Host-side counts: live entries, deleted slots, capacity (each may be NULL). */
mg_status_t mg_hash_info(mg_hash_t H, int64_t* size, int64_t* deleted, int64_t* capacity);

/* 128-bit Morton keys (B = 42): d_ijk [n][3] int64 coordinates in [0, 2^42)
 * -> d_keys [n][2] uint64 (low word, high word).  Asynchronous on `stream`. */
mg_status_t mg_op_morton128(int64_t n, const int64_t* d_ijk, uint64_t* d_keys, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MG_H_ */

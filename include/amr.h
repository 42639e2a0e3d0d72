/*
 * libamr -- MI355X (gfx950) AMR compressible-Euler hot path, C ABI.
 *
 * The library advances the compressible Euler equations (Section 2.1 of
 * "Task-Based Programming for Adaptive Mesh Refinement in Compressible Flow
 * Simulations", Eq. (1)-(7); calorically perfect gas, R = 1) on a forest of
 * equal-shape patches (Section 3.2) that obeys the validity rules R1/R2 and is
 * adapted by the recursive refinement and the coarsening procedures of
 * Section 3.3 (Algorithms 1 and 2).  Fluxes are WENO5-JS interpolated
 * primitives (p, T, u_j) combined by the Rusanov solver (Eq. (10)-(12)); the
 * divergence is the 4th-order staggered difference of Eq. (9), written in
 * conservative face-flux form; time advancement is SSP-RK3 (Section 2.2).
 * All solution arithmetic is FP64.
 *
 * Conventions shared by every call
 *  - Patch data are cell-centred.  A patch of level l has n_l cells per
 *    dimension plus ng = 4 ghost layers on every side; its storage is
 *    structure-of-arrays, var-major: [var][z][y][x] over the full
 *    (n_l + 8)^dim box, x fastest.  Variables are (rho, rho u_x[, rho u_y
 *    [, rho u_z]], rho e).
 *  - "pid" is a patch slot index in [0, max_patches).  Slots are partitioned
 *    by level; a pid's level never changes while it is active.
 *  - State buffers: 0 = U^n, 1 = A, 2 = B (the two SSP-RK3 stage buffers).
 *  - Calls marked "async" enqueue work on the hierarchy's HIP stream and
 *    return; calls marked "sync" wait for that stream before returning.
 *  - Device pointers ("_dev") are caller-owned device memory; host pointers
 *    ("_host") are caller-owned host memory.  The library never frees either.
 *  - Every call returns an amr_status; on failure amr_last_error() gives a
 *    message.  No C++ exception crosses this interface.  A hierarchy is not
 *    re-entrant: one thread (and one stream) per hierarchy.
 */
#ifndef AMR_H
#define AMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amr_hierarchy amr_hierarchy;

typedef enum {
  AMR_OK = 0,
  AMR_E_ARG = -1,          /* invalid argument or configuration */
  AMR_E_CAPACITY = -2,     /* patch pool exhausted; hierarchy unchanged */
  AMR_E_HIP = -3,          /* a HIP runtime call failed */
  AMR_E_MESH = -4,         /* R1/R2 or a ghost/prolongation source missing */
  AMR_E_NONPHYSICAL = -5,  /* rho <= 0, p <= 0 or NaN in a leaf cell */
  AMR_E_STATE = -6         /* call not valid in the current state */
} amr_status;

enum { AMR_MAX_LEVELS = 8, AMR_GHOST = 4 };
enum { AMR_EXEC_PER_PATCH = 0, AMR_EXEC_BATCHED = 1 };
enum { AMR_COARSEN_TEXT = 0, AMR_COARSEN_LITERAL = 1 };
/* Interpolation of the edge states (Section 2.2): WENO5-JS on the primitive
 * set (p, T, u_j); the 4th-order central interpolation of Eq. (8) (shock-free
 * flows); WENO5-JS on characteristic variables (the eigenvectors of the
 * direction's flux Jacobian at the mean of the two nodes beside the edge). */
enum { AMR_SCHEME_WENO = 0, AMR_SCHEME_CENTRAL = 1, AMR_SCHEME_CHAR = 2 };

/* Optional device allocator (e.g. a framework's caching allocator).  alloc
 * returns device memory of at least `bytes` bytes aligned to 256 B, or NULL. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} amr_allocator;

/* Run configuration (Section 3.2: fixed-capacity patch pool `np_max`, patch
 * size, ghost width; Section 5: gamma, R = 1, CFL). */
typedef struct {
  int dim;                           /* 1, 2 or 3 */
  int max_levels;                    /* 1 .. AMR_MAX_LEVELS */
  int base_cells;                    /* level-0 cells per dimension */
  int patch_cells[AMR_MAX_LEVELS];   /* patch edge n_l; even, >= 4; n_{l+1} | 2 n_l */
  int periodic[3];                   /* per dimension: 1 periodic, 0 transmissive */
  double lo, hi;                     /* domain [lo, hi)^dim */
  double gamma;                      /* ratio of specific heats (1.4) */
  double cfl;                        /* dt = cfl / max_leaf sum_j (|u_j| + c) / h_l */
  double weno_eps;                   /* WENO5-JS epsilon (1e-6), in [1e-20, 1] */
  double tag_theta;                  /* gradient tag threshold (0.02) */
  int tag_buffer;                    /* tag dilation in cells (0 .. 3) */
  int max_patches;                   /* total patch slots over all levels */
  int level_capacity[AMR_MAX_LEVELS];/* slots per level; 0 = derive from max_patches */
  int exec_mode;                     /* AMR_EXEC_PER_PATCH or AMR_EXEC_BATCHED */
  int coarsen_rule;                  /* AMR_COARSEN_TEXT (default) or _LITERAL */
  int scheme;                        /* AMR_SCHEME_WENO (default), _CENTRAL or _CHAR */
} amr_config;

/* One row of the patch table (Fig. grid-meta of the paper: level, nbr,
 * parent, child, plus the patch position). */
typedef struct {
  int32_t pid;
  int32_t level;
  int32_t coord[3];      /* patch position on its level, (x, y, z) */
  int32_t parent;        /* -1 on level 0 */
  int32_t nchildren;     /* 0 for a leaf */
  int32_t first_child;   /* lowest child pid, -1 for a leaf */
  int32_t nbr[26];       /* Moore neighbours in (dz, dy, dx) lexicographic
                            order, dx fastest, centre skipped; 3^dim - 1
                            entries used; -1 = absent or physical boundary */
} amr_patch_info;

/* Create a hierarchy holding every level-0 patch (sync).  `alloc` may be
 * NULL (hipMalloc is used); `hip_stream` may be NULL (default stream).
 * Device memory: 3 state buffers, one flux-register pool and the tables,
 * all sized from max_patches so that regridding never reallocates.
 * Errors: AMR_E_ARG for an invalid config, AMR_E_HIP on allocation failure;
 * on failure *out still receives an object whose amr_last_error() explains
 * the failure and which must be passed to amr_destroy_hierarchy. */
amr_status amr_create_hierarchy(const amr_config* cfg, const amr_allocator* alloc,
                                void* hip_stream, amr_hierarchy** out);
amr_status amr_destroy_hierarchy(amr_hierarchy* h);
const char* amr_last_error(const amr_hierarchy* h);

/* Sizes and layout queries (no device work).  amr_patch_offset gives the
 * state offset of a patch's box; the first level's pool starts after a head
 * pad of a few doubles (a multiple of nvar) that puts every interior row of
 * a box, for n_l a multiple of 8, on a 64-byte boundary of a
 * 256-byte-aligned buffer. */
amr_status amr_num_patches(const amr_hierarchy* h, int* nactive, int* nleaf);
amr_status amr_patch_doubles(const amr_hierarchy* h, int level, int64_t* n);
amr_status amr_state_doubles(const amr_hierarchy* h, int64_t* n);
amr_status amr_patch_offset(const amr_hierarchy* h, int pid, int64_t* off);
amr_status amr_state_ptr(const amr_hierarchy* h, int buf, double** dev);

/* Active patches sorted by (level, z, y, x); writes at most `cap` rows and
 * the total count to *n (sync). */
amr_status amr_get_patch_table(const amr_hierarchy* h, amr_patch_info* out, int cap, int* n);

/* Upload / download whole patch arrays (ghosts included) for `npatch` pids;
 * the host buffer is the concatenation of the patches' arrays in `pids`
 * order (sync); patches adjacent in their level's pool move in one copy.
 * amr_set_state_prim takes interior primitive values (rho, u_x[, u_y[,
 * u_z]], p), var-major over n_l^dim cells per patch, converts them on the
 * device to rho, rho u and E = p / (gamma - 1) + rho u.u / 2 (Eq. (4), (6))
 * and leaves ghost cells as they are; it stages the values through a device
 * buffer of at most 128 MiB (or one patch), taken from the hierarchy's
 * allocator and returned before it returns.  Each pid appears at most
 * once.  An inactive pid is AMR_E_ARG, found before anything is written. */
amr_status amr_set_state(amr_hierarchy* h, int buf, const double* host, const int* pids, int npatch);
amr_status amr_get_state(const amr_hierarchy* h, int buf, double* host, const int* pids, int npatch);
amr_status amr_set_state_prim(amr_hierarchy* h, int buf, const double* host_prim,
                              const int* pids, int npatch);

/* amr_set_state_prim for callers that cannot allocate device memory (code
 * under HIP graph capture excepted: the call copies from host memory and
 * waits): the same conversion and result, staged through a fixed per-GPU
 * scratch array of AMR_NOALLOC_SCRATCH_BYTES that the library holds from
 * its first hierarchy on that GPU until the process ends, instead of a
 * buffer from the allocator; no hipMalloc, hipFree or allocator call.
 * One call takes at most AMR_NOALLOC_SCRATCH_BYTES of primitives and patch
 * indices (8 bytes per interior value, rounded up to 256 bytes, plus 12
 * bytes per patch); a larger call is AMR_E_ARG before anything is copied
 * (split the patches over several calls).  Sync.  Every hierarchy on one GPU
 * shares that GPU's scratch, so calls that overlap in time on one GPU (from
 * several host threads) race; calls from one thread never overlap. */
enum { AMR_NOALLOC_SCRATCH_BYTES = 32 << 20 };
amr_status amr_set_state_prim_noalloc(amr_hierarchy* h, int buf, const double* host_prim,
                                      const int* pids, int npatch);

/* Ghost fill of every active patch of buffer `buf` (async): same-level
 * source where an active same-level patch covers the (wrapped or clamped)
 * ghost position, otherwise conservative MC-limited linear prolongation
 * from the level below (multi-resolution support required by R2). */
amr_status amr_fill_ghosts(amr_hierarchy* h, int buf);

/* L(U) of buffer `buf` on every leaf patch (async), including the
 * coarse/fine flux correction: Section 2.2 fluxes and Eq. (9) divergence.
 * The ghost cells the stencils read are filled first (with the fused halo,
 * the default, only the prolonged cells of the face ghost regions: the
 * stencils are one-directional, so edge and corner ghost regions keep their
 * previous contents; amr_fill_ghosts fills them all).  rhs_dev has
 * amr_state_doubles() entries in the state-buffer layout; leaf interiors
 * are written. */
amr_status amr_rhs(amr_hierarchy* h, int buf, double* rhs_dev);

/* dt = cfl / max over leaf cells of buffer `buf` of sum_j (|u_j| + c) / h_l,
 * with c from Eq. (7); written to the device scalar *dt_dev (async). */
amr_status amr_compute_dt(amr_hierarchy* h, int buf, double* dt_dev);

/* One SSP-RK3 stage (1, 2 or 3; async): fill the ghosts of the stage input
 * that the stencils read (as amr_rhs), fused RHS + stage combination on
 * every leaf (tiles of the finest level also restrict themselves into their
 * parents), coarse/fine flux correction, restriction of every other
 * non-leaf patch.  dt is read from the device scalar. */
amr_status amr_rk_stage(amr_hierarchy* h, int stage, const double* dt_dev);

/* dt (into *dt_dev) followed by the three stages (async).  In batched mode
 * dt is computed inside the first stage's launch from the CFL rate the
 * previous step's last stage accumulated (or a fresh one after a regrid). */
amr_status amr_step(amr_hierarchy* h, double* dt_dev);

/* Gradient tagging of buffer `buf` (async; halo cells come from the
 * same-level neighbours, or from ghost layers filled first when the fused halo
 * is off; prolonged ghost cells are always filled first).
 * Per pid (max_patches entries each): refine_req = leaf below the finest
 * level with a tagged cell within tag_buffer cells of its interior;
 * coarsen_req = patch whose children are all leaves without tags and whose
 * own (restricted) data carry no tag either (the requests of Fig.
 * grid-meta; the tag criterion itself is not given in the paper).  cell_tags_dev (nullable) receives the
 * dilated per-cell tag of every leaf interior cell, one byte per cell in a
 * layout of (n_l + 8)^dim bytes per patch at offset amr_patch_offset/nvar. */
amr_status amr_tag(amr_hierarchy* h, int buf, uint8_t* refine_req_dev,
                   uint8_t* coarsen_req_dev, uint8_t* cell_tags_dev);

/* Apply refinement (Algorithm 1, recursive) then coarsening (Algorithm 2)
 * requests given per pid on the host (sync).  New patches of U^n are
 * prolonged from the level below.  Transactional: on AMR_E_CAPACITY the mesh
 * is unchanged.  *ncreated / *ndeleted may be NULL. */
amr_status amr_regrid(amr_hierarchy* h, const uint8_t* refine_req_host,
                      const uint8_t* coarsen_req_host, int* ncreated, int* ndeleted);

/* amr_tag on U^n followed by amr_regrid with those requests (sync). */
amr_status amr_adapt(amr_hierarchy* h, int* ncreated, int* ndeleted);

/* Count leaf cells of U^n with rho <= 0, p <= 0 or NaN (sync); returns
 * AMR_E_NONPHYSICAL when the count is positive. */
amr_status amr_check(amr_hierarchy* h, int* nonphysical_count);

/* Pids created by the most recent regrid, in creation order (no device work). */
amr_status amr_last_created(const amr_hierarchy* h, int* pids, int cap, int* n);

/* Reads and clears the sticky ghost-fill/prolongation error flag: 1 when a
 * fill or the prolongation of a new patch found no same-level or coarser
 * source (an invalid mesh) since the flag was last read (sync). */
amr_status amr_fill_error(amr_hierarchy* h, int* flag);

/* Host-only replay of mesh adaptation, for checking the refinement and
 * coarsening procedures without a GPU (no device work).  `req` holds `nreq`
 * records of 6 int32: (round, kind, level, x, y, z) with kind 0 = refine
 * request, 1 = coarsen request, sorted by round; each round's requests are
 * applied as one regrid (Algorithm 1 then Algorithm 2) to a fresh base mesh.
 * Requests naming an inactive position are ignored.  The resulting active
 * patches are returned as by amr_get_patch_table (nbr not filled). */
amr_status amr_forest_replay(const amr_config* cfg, const int32_t* req, int nreq,
                             amr_patch_info* out, int cap, int* n);

/* Velocity-gradient diagnostic (the velocity-gradient task of the paper's
 * fusion listing, §4.1, whose body the paper elides; the numerical Schlieren
 * images of §5 are drawn from the density gradient).  Ghosts of the leaves
 * of `buf` are filled first; then at every interior cell of every leaf
 * patch, with u_i = m_i / rho and h the cell's level spacing:
 *   G[i][j] = (u_i(x + h e_j) - u_i(x - h e_j)) / (2h)   (component i*d + j)
 *   S = sqrt(sum_j ((rho(x + h e_j) - rho(x - h e_j)) / (2h))^2)  (component d*d)
 * out_dev (caller-owned device memory) holds d*d + 1 planes of
 * amr_state_doubles() / (d + 2) doubles each; a plane has the cell layout of
 * one variable of the state buffer (a patch's (n+8)^d box starts at the
 * patch's state offset divided by d + 2).  Only leaf interior cells are
 * written.  Async on the hierarchy's stream. */
amr_status amr_velocity_gradient(amr_hierarchy* h, int buf, double* out_dev);

/* Number of leaf cells (sum of n_l^dim over leaf patches) of the current
 * mesh (no device work): the cells one step advances. */
amr_status amr_leaf_cells(const amr_hierarchy* h, int64_t* cells);

/* Timing of the fused RHS + stage kernel: while enabled, every launch of it
 * carries a pair of HIP events that the dispatch itself stamps at its start
 * and end (extended launch), and amr_step launches eagerly.  amr_profile
 * (sync) enables/disables and resets; amr_profile_read (sync) returns the
 * summed event time in ms, the number of launches and the leaf cells they
 * covered. */
amr_status amr_profile(amr_hierarchy* h, int enable);
amr_status amr_profile_read(amr_hierarchy* h, double* total_ms, int* launches, int64_t* cells);

/* The plain tagger as judge (sync): *uncovered = number of leaves below the
 * finest level that the gradient tagger would refine now on U^n (0 = the
 * current mesh covers every tag). */
amr_status amr_judge(amr_hierarchy* h, int* uncovered);

/* Tag dilation (amr_config.tag_buffer, 0..3 cells) for the following tag,
 * adapt and judge calls (no device work); AMR_E_ARG outside 0..3.  Lets a
 * caller regrid with a wider dilation than its judge checks coverage with. */
amr_status amr_set_tag_buffer(amr_hierarchy* h, int cells);

/* Execution mode switch (AMR_EXEC_PER_PATCH launches one kernel per patch per
 * phase; AMR_EXEC_BATCHED launches each phase once over all patches). */
amr_status amr_set_exec_mode(amr_hierarchy* h, int mode);

/* ------------------------------------------------------------------------
 * Learned refinement predictor (2D and 3D; not part of the paper).  A
 * convolutional network forecasts which cells the gradient tagger will tag
 * within the next steps, so that regridding can run less often; the plain
 * tagger remains the judge.  BF16 weights and activations, FP32 accumulation
 * (MFMA).  Training: weighted binary cross-entropy with logits averaged over
 * cells, gradients reduced over tiles in a fixed order, Adam (beta 0.9 /
 * 0.999, eps 1e-8) on the FP32 master weights followed by a
 * round-to-nearest-even BF16 copy.
 *
 * 2D (one tile = one patch of edge n = patch_cells, 8..32, even): input
 * normalised (rho, u, v, p) of the patch plus 3 halo cells, pixel-major with
 * 4 channels innermost ([ntile][(n+6)^2][4]); three valid 3x3 convolutions
 * 4 -> 16 -> 16 -> 1, bias, ReLU after the first two; logits [ntile][n^2].
 * Parameters (3057 floats): W1 [16][4][3][3], b1 [16], W2 [16][16][3][3],
 * b2 [16], W3 [16][3][3], b3.
 *
 * 3D (tiles of 8^3 cells; patch_cells must be 8): input normalised
 * (rho, u, v, w, p) of the tile plus 3 halo cells, voxel-major with 8
 * channels innermost, the last 3 zero ([ntile][14^3][8]); three valid 3x3x3
 * convolutions 5 -> 8 -> 8 -> 1; logits [ntile][8^3] (z, y, x order).
 * Parameters (3041 floats): W1 [8][5][3][3][3], b1 [8], W2 [8][8][3][3][3],
 * b2 [8], W3 [8][3][3][3], b3.  Prediction covers every leaf whose edge is a
 * multiple of 8, tile by tile.
 * ---------------------------------------------------------------------- */
typedef struct amr_cnn amr_cnn;
typedef struct {
  int patch_cells;   /* 2D: leaves whose edge is n are predicted; 3D: 8 */
  float mean[5];     /* normalisation of (rho, u, v, p) in 2D, (rho, u, v, w, p) in 3D */
  float std[5];
  float pos_weight;  /* weight of the positive class in the loss */
  int max_batch;     /* tiles per forward/training call (1..4096) */
} amr_cnn_config;

/* Buffers of the predictor come from the hierarchy's allocator (sync). */
amr_status amr_cnn_create(amr_hierarchy* h, const amr_cnn_config* cfg, amr_cnn** out);
amr_status amr_cnn_destroy(amr_cnn* c);
amr_status amr_cnn_num_params(const amr_cnn* c, int* n);
/* FP32 master weights from / to the host (sync); setting resets Adam. */
amr_status amr_cnn_set_weights(amr_cnn* c, const float* host_fp32, int n);
amr_status amr_cnn_get_weights(amr_cnn* c, float* host_fp32, int n);
/* Input tiles of the given leaf pids (patches of edge patch_cells, one tile
 * each) of buffer `buf` (ghosts filled first) into x_dev (sync). */
amr_status amr_cnn_gather(amr_cnn* c, int buf, const int* pids_host, int npatch, uint16_t* x_dev);
/* Logits of npatch <= max_batch input tiles (async). */
amr_status amr_cnn_forward(amr_cnn* c, const uint16_t* x_dev, int npatch, float* logits_dev);
/* Forward, loss (-> *loss_dev), backward; if lr > 0 one Adam step (async).
 * labels_dev: [npatch][n^d] bytes (0/1); grads_dev (nullable) receives the
 * summed parameter gradient. */
amr_status amr_cnn_train_step(amr_cnn* c, const uint16_t* x_dev, const uint8_t* labels_dev,
                              int npatch, float lr, float* loss_dev, float* grads_dev);
/* Predicted requests on buffer `buf` (sync): a predicted leaf is flagged when
 * any of its cells has probability > tau; refine_req = flagged leaves below the
 * finest level, coarsen_req = patches whose children are all unflagged
 * leaves (both per pid, max_patches bytes, device). */
amr_status amr_cnn_predict(amr_cnn* c, int buf, float tau, uint8_t* refine_req_dev,
                           uint8_t* coarsen_req_dev);
/* D = A B for 16x16 BF16 matrices on one wave (checks the MFMA lane layout
 * the predictor kernels assume; async). */
amr_status amr_cnn_mfma_selftest(amr_hierarchy* h, const uint16_t* a_dev, const uint16_t* b_dev,
                                 float* d_dev);

/* hipGraph replay of amr_step in batched mode (default off): the kernels of
 * one step are captured once (two graphs, one per CFL-rate slot) and
 * replayed; the graph holds kernel nodes only.  Batched launches of the
 * step's kernels read their work lists and live counts from a device list
 * directory that regrids rewrite, and after a regrid that changes the mesh
 * the next replay first sets the grid of each list launch in the
 * instantiated graph to the list's new length, so regrids never record the
 * graphs again (with the fused halo off, the explicit ghost fill is sized by
 * the leaf count and every mesh change re-records them).  A change of tile
 * variant, execution mode, halo mode, tag dilation or dt pointer re-records
 * them.  Enabling an enabled graph mode keeps the recorded graphs.  Results
 * are identical to eager launches. */
amr_status amr_set_graph(amr_hierarchy* h, int enable);
/* Number of step graphs recorded since creation (test and profiling hook). */
amr_status amr_graph_records(const amr_hierarchy* h, int* recorded);

/* Tile variants of the fused stage kernel (cells per tile and block size):
 * 0: 16 (1D, 64 threads), 1: 8 (1D), 2: 16x16 (2D, 320), 3: 16x8 (2D, 192),
 * 4: 8x8 (2D, 128), 5: 8x8x8 (3D, 768), 6: 8x8x4 (3D, 448), 7: 4x4x4 (3D, 128);
 * 8, 9, 10: 16x16, 16x8, 8x8 (2D) computing the x and y edge fluxes in one
 * sweep (more LDS, fewer block barriers).
 * A variant is admissible when its extents divide every level's patch edge.
 * Every variant performs the same operations per cell: results are
 * identical.  amr_set_tile_variant (sync) selects one; amr_autotune (sync)
 * times `reps` launches of each admissible variant on the current mesh
 * (writing the stage buffer B and the flux registers) and keeps the fastest. */
amr_status amr_set_tile_variant(amr_hierarchy* h, int variant);
amr_status amr_get_tile_variant(const amr_hierarchy* h, int* variant, int* tx, int* ty, int* tz,
                                int* threads);
amr_status amr_autotune(amr_hierarchy* h, int reps, int* best, float* best_ms);

/* Halo source of the fused stage kernel: 1 (default) reads halo nodes that
 * lie in same-level neighbours straight from those neighbours, and only the
 * ghost cells that need prolongation are filled beforehand (over the ghost
 * regions without a same-level source); 0 runs the full fill kernel first
 * and reads the filled ghost layers.  Results are identical. */
amr_status amr_set_fused_halo(amr_hierarchy* h, int enable);

#ifdef __cplusplus
}
#endif
#endif /* AMR_H */

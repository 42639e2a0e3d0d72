// Internal structures shared by the host mesh manager, the kernels and the
// C-ABI layer of libamr.  Not part of the public interface (include/amr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/amr.h"

namespace amr {

constexpr int kNG = AMR_GHOST;   // ghost layers (flux-form Eq. (9) + WENO5 need 4)
constexpr int kMaxLev = AMR_MAX_LEVELS;

// Per-level constants, mirrored on the device by value.
// XCDs of the MI355X (gfx950): 8 dies of 32 compute units, one L2 each.
constexpr int kXcds = 8;

struct LevelC {
  int n;             // patch edge (cells)
  int full;          // n + 2 ng
  int np;            // patches per dimension on this level
  int cells;         // cells per dimension on this level
  int pid_base;      // first pid of this level's slot range
  int cap;           // slots of this level
  int map_off;       // offset of this level's patch map (np^dim ints)
  int ratio;         // children per dimension (2 n_l / n_{l+1}); 0 on the finest level
  long long pool_off;  // offset (doubles) of this level's pool in a state buffer
  long long stride;    // doubles per patch (nvar * full^dim)
  long long fr_off;    // offset (doubles) of this level's flux-register pool
  long long fr_stride; // doubles per patch of flux registers (2 dim nvar n^(dim-1))
  long long tag_off;   // offset (bytes) of this level's cell-tag pool
  double h, inv_h;
};

// Everything a kernel needs to address patch data, passed by value.
struct DevMesh {
  int dim, nvar, nlev, scheme;
  int tile;           // stage-kernel tile variant (index into Kernels::variant)
  int periodic[3];
  int max_patches, maxc;
  double gamma, gm1, igm1, eps, theta, cfl;
  int tag_buffer;
  LevelC lv[kMaxLev];
  const int* level;    // [max_patches]
  const int* coord;    // [max_patches * 3]
  const int* parent;   // [max_patches]
  const int* nchild;   // [max_patches]
  const int* child;    // [max_patches * maxc]
  const int* map;      // all levels' patch maps
};

// Work lists, all resident in one device int buffer.  `dir` (null for lists
// outside it) is the list's entry {offset into the buffer, count} of the
// device list directory, which batched launches of the step's kernels read
// at run time, so that a recorded step stays valid across regrids as long
// as each list fits the grid it was recorded with.
struct ListView {
  const int* ptr;
  int count;
  const int* dir = nullptr;
};

// Launch wrappers implemented in kernels.hip.
struct Kernels {
  // coarse_only: write only the ghost cells without a same-level source
  // (the prolonged ones)
  static void fill(const DevMesh& m, double* U, const int* list, int count, int* err,
                   bool coarse_only, hipStream_t s);
  // prolonged ghost cells only, over (pid, ghost region) pairs
  // dir (nullable): list directory entry; with it `list` is the list buffer
  // and the list and its live count are read at run time, and `count` only
  // sizes the grid (at least the live count: one block per item)
  // Grids (blocks) of the batched launches for a list of `count` items, for
  // updating the launches of a recorded step graph after a regrid.
  static int fill_cf_grid(const DevMesh& m, int count);
  static int stage_grid(int count) { return ((count + kXcds - 1) / kXcds) * kXcds; }
  static void fill_cf(const DevMesh& m, double* U, const int* list, int count, const int* dir,
                      int* err, hipStream_t s);
  // fuse = halo nodes outside the patch with a same-level source are read
  // from that source by the kernel itself; the others (prolonged) come from
  // ghost layers filled before by fill_cf
  // lam_next (nullable, stage 3 only): accumulate the next step's CFL rate
  // over leaf cells not on coarse/fine faces (cfmask: per-pid face bits)
  // ev0/ev1 (optional): events stamped at the dispatch's own start and end.
  // lam_in (stage 1 only, optional): take dt = CFL / *lam_in instead of *dt,
  // write it to *dt_out and clear *lam_next (the slot stage 3 accumulates in)
  // In the stage modes a tile of the finest level (nlev - 1 >= 1) also
  // restricts its new values into its parent patch.
  static void stage(const DevMesh& m, int mode, const double* Uin, const double* Un,
                    double* out, double* fr, const int* tiles, int count, const int* dir,
                    const double* dt, bool fuse, unsigned long long* lam_next,
                    const uint8_t* cfmask, hipStream_t s, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr, const unsigned long long* lam_in = nullptr,
                    double* dt_out = nullptr);
  static void reflux(const DevMesh& m, int mode, double* out, const double* fr,
                     const int* list, int count, const double* dt, double w,
                     unsigned long long* lam_next, hipStream_t s);
  // refluxing and the restriction of the two finest levels in one launch:
  // reflux items, level-lup patches with children (plist), level-lup leaves
  // without coarse/fine faces (slist); lup = finest level - 1
  // dir (nullable): the directory entries of the three lists, in order;
  // with it the list pointers are the list buffer, the live counts are read
  // at run time and nref + npair + nsingle only sizes the grid.
  // fine_done: the stage kernel has already restricted the finest level.
  static void post(const DevMesh& m, int mode, double* out, const double* fr, const int* rlist,
                   int nref, const int* plist, int npair, const int* slist, int nsingle,
                   const int* dir, int lup, bool fine_done, const double* dt, double w,
                   unsigned long long* lam_next, hipStream_t s);
  static void restrict_level(const DevMesh& m, double* U, const int* list, int count,
                             const int* dir, hipStream_t s);
  static void max_rate(const DevMesh& m, const double* U, const int* list, int count,
                       unsigned long long* lam_bits, hipStream_t s);
  static void zero_u64(unsigned long long* p, hipStream_t s);
  // dt = cfl / rate; also zeroes *clear (nullable), the next rate accumulator
  static void dt_from_rate(const DevMesh& m, const unsigned long long* lam_bits,
                           double* dt, unsigned long long* clear, hipStream_t s);
  // fuse: halo cells read from same-level neighbours directly; ghost layers
  // hold only the prolonged cells (filled by fill_cf beforehand)
  static void tag(const DevMesh& m, const double* U, const int* list, int count,
                  uint8_t* has_tag, uint8_t* raw, bool fuse, hipStream_t s);
  static void cell_tags(const DevMesh& m, const uint8_t* raw, const int* list, int count,
                        uint8_t* out, hipStream_t s);
  static void requests(const DevMesh& m, const uint8_t* has_tag, const uint8_t* active_leaf,
                       int nslots, uint8_t* refine, uint8_t* coarsen, hipStream_t s);
  static void prolong_new(const DevMesh& m, double* U, const int* list, int count, int* err,
                          hipStream_t s);
  static void scatter_int(int* dst, const int* pairs, int npairs, hipStream_t s);
  static void count_nonzero(const uint8_t* a, int n, int* out, hipStream_t s);
  static void check(const DevMesh& m, const double* U, const int* list, int count,
                    int* bad, hipStream_t s);
  // Tile variants of the stage kernel: extents (cells) and block size.
  struct TileVariant {
    int dim, tx, ty, tz, threads;
    int both = 0;  // 2D: x and y edges computed in one sweep
  };
  static int num_variants();
  static TileVariant variant(int v);
  // Whether variant v fits every level's patch edge.
  static bool variant_fits(int v, int dim, const int* n, int nlev);
  // First fitting variant of a dimension (the default), -1 when none fits.
  static int default_variant(int dim, const int* n, int nlev);
  static int tiles_per_patch(int v, int n);
};

// Stage modes of the fused RHS/combine kernel.
enum StageMode { kModeRHS = 0, kModeStage1 = 1, kModeStage2 = 2, kModeStage3 = 3 };

}  // namespace amr

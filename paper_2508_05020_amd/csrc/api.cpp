// C-ABI layer of libamr: the hierarchy object, device tables and work lists,
// and the sequencing of the kernels for each call of include/amr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "amr_internal.hpp"
#include "forest.hpp"
#include "cnn_internal.hpp"
#include "diag_internal.hpp"
#include "state_io_internal.hpp"

namespace {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct StateError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIP_OK(expr)                                                         \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      std::ostringstream os_;                                                \
      os_ << #expr << ": " << hipGetErrorString(e_);                         \
      throw HipError(os_.str());                                             \
    }                                                                        \
  } while (0)

// entries of the device list directory
enum { kDirCf = 0, kDirTiles = 1, kDirReflux = 2, kDirPairs = 3, kDirSingles = 4, kDirCfFace = 5,
       kDirRestr = 6, kDirEntries = kDirRestr + amr::kMaxLev };

}  // namespace

struct amr_hierarchy {
  amr_config cfg{};
  amr::Forest forest;
  amr::DevMesh dm{};
  hipStream_t stream = nullptr;
  // device address of the staging array of amr_set_state_prim_noalloc on this
  // hierarchy's device (resolved at creation)
  void* noalloc_scratch = nullptr;
  amr_allocator alloc{};
  bool has_alloc = false;
  std::string err;
  int nvar = 0;
  int exec_mode = AMR_EXEC_BATCHED;
  bool fuse_halo = true;  // stage kernel gathers halos itself (no fill pass)
  // hipGraphs of one batched step (dt + 3 stages), one per parity of the CFL
  // rate double buffer.  Their launches read the work lists and live counts
  // from the list directory; after a regrid that changes the mesh the grid
  // of each list launch is set to its new list length in the instantiated
  // graph (gnodes: the launch nodes and the lists that size them, noted
  // while recording), so a regrid never records them again.  A tile, mode
  // or configuration change does.
  struct GridNode {
    hipGraphNode_t node;
    int kind;        // kGn* below
    int e[3], ne;    // directory entries whose counts add up to the items
    int grid;        // blocks in the instantiated graph
  };
  bool use_graph = false;
  bool capturing = false;
  int cap_slot = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t step_graph[2] = {nullptr, nullptr};
  hipGraphExec_t step_exec[2] = {nullptr, nullptr};
  const double* step_exec_dt[2] = {nullptr, nullptr};
  bool step_exec_valid = false;
  bool step_exec_ok[2] = {false, false};
  std::vector<GridNode> gnodes[2];
  long long mesh_version = 0;          // sync_tables calls so far
  long long rec_version[2] = {-1, -1};  // mesh_version the graphs' grids match
  int step_records = 0;  // step graphs recorded so far
  // CFL rate of U^n: slot lam_cur holds it when lam_valid; the step being
  // run accumulates the next one into the other slot (slot 2: amr_compute_dt)
  int lam_cur = 0;
  bool lam_valid = false;
  uint8_t* d_cfmask = nullptr;
  std::vector<void*> owned;

  // device memory
  double* U[3] = {nullptr, nullptr, nullptr};
  long long state_doubles = 0;
  double* fr = nullptr;
  long long fr_doubles = 0;
  long long tag_bytes = 0;
  int* d_tab = nullptr;  // level | parent | nchild | coord | child | map
  long long tab_ints = 0;
  long long off_level = 0, off_parent = 0, off_nchild = 0, off_coord = 0, off_child = 0,
            off_map = 0;
  uint8_t* d_active_leaf = nullptr;
  uint8_t* d_has_tag = nullptr;
  uint8_t* d_raw = nullptr;
  uint8_t* d_refine = nullptr;
  uint8_t* d_coarsen = nullptr;
  unsigned long long* d_lam = nullptr;
  double* d_dt = nullptr;
  int* d_flags = nullptr;  // [0] fill/prolong error, [1] nonphysical count
  int* d_lists = nullptr;
  long long lists_cap = 0;
  // list directory: {offset into d_lists, count} of the lists the step's
  // kernels take (entries kDirCf, kDirTiles, kDirReflux, kDirPairs,
  // kDirSingles, kDirRestr + level), rewritten with the lists; batched
  // launches read it, so a recorded step survives a regrid
  int* d_dir = nullptr;
  int* h_dir = nullptr;  // pinned staging of the directory
  int* d_pairs = nullptr;
  long long pairs_cap = 0;
  // pinned host staging for table/list uploads (reused; every regrid first
  // drains the stream, so earlier copies from it have completed)
  char* h_stage = nullptr;
  size_t h_stage_bytes = 0;
  uint8_t* h_req = nullptr;  // pinned: refine and coarsen requests read back by amr_adapt

  // host mirrors of the work lists
  std::vector<int> lists;
  // cffaces: the face regions of cfregions (all the stage kernel reads;
  // the tagger's dilated box reads the edge and corner regions too)
  amr::ListView all{}, leaves{}, tiles{}, reflux{}, cfregions{}, cffaces{}, cands{};
  // post-stage restriction of the two finest levels (see Kernels::post)
  amr::ListView post_pairs{}, post_singles{};
  amr::ListView restr[amr::kMaxLev]{}, fresh[amr::kMaxLev]{};
  std::vector<int> last_created;
  // scratch of sync_tables, per parent: all Moore neighbours have children;
  // bit mask (offset codes) of the Moore neighbours with children
  std::vector<int8_t> parent_interior;
  std::vector<int> parent_kids;
  std::vector<uint8_t> h_active_leaf;
  long long leaf_cells = 0;

  // optional timing of the fused stage kernel with HIP events
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<long long> ev_cells;
  // A pair of events for one profiled launch; the launch stamps them itself
  // at its start and end, so the interval is the kernel's own duration.
  void prof_pair(hipEvent_t* a, hipEvent_t* b, long long cells) {
    if (ev_used + 2 > ev_pool.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        ev_pool.push_back(e);
      }
    }
    *a = ev_pool[ev_used++];
    *b = ev_pool[ev_used++];
    ev_cells.push_back(cells);
  }

  void* dev_alloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    if (has_alloc) {
      p = alloc.alloc(bytes, alloc.ctx);
      if (!p) throw HipError("device allocator returned NULL");
      // kernels load aligned pairs of doubles as 16-byte vectors
      if (reinterpret_cast<uintptr_t>(p) & 255) {
        alloc.free(p, alloc.ctx);
        throw ArgError("device allocator returned memory not aligned to 256 B");
      }
    } else {
      HIP_OK(hipMalloc(&p, bytes));
    }
    owned.push_back(p);
    return p;
  }
  // frees one allocation made by dev_alloc before the hierarchy ends
  void dev_free(void* p) {
    auto it = std::find(owned.begin(), owned.end(), p);
    if (it == owned.end()) return;
    owned.erase(it);
    if (has_alloc) alloc.free(p, alloc.ctx);
    else (void)hipFree(p);
  }
  void release_all() {
    for (int k = 0; k < 2; ++k) {
      if (step_exec[k]) (void)hipGraphExecDestroy(step_exec[k]);
      step_exec[k] = nullptr;
      if (step_graph[k]) (void)hipGraphDestroy(step_graph[k]);
      step_graph[k] = nullptr;
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
    if (h_stage) (void)hipHostFree(h_stage);
    h_stage = nullptr;
    if (h_req) (void)hipHostFree(h_req);
    h_req = nullptr;
    if (h_dir) (void)hipHostFree(h_dir);
    h_dir = nullptr;
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    ev_pool.clear();
    for (void* p : owned) {
      if (has_alloc) alloc.free(p, alloc.ctx);
      else (void)hipFree(p);
    }
    owned.clear();
  }
  void check_launch() { HIP_OK(hipGetLastError()); }
  void sync() { HIP_OK(hipStreamSynchronize(stream)); }
};

namespace {

using amr::Kernels;

int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// staging of amr_set_state_prim: at most 16 Mi doubles (128 MiB, or one patch
// if larger) and 64 Ki patches per batch
constexpr long long kPrimStageDoubles = 16LL << 20;
constexpr long long kPrimStagePatches = 65536;

// one contiguous copy: device offset, host offset, doubles
struct CopyRun {
  long long dev, host, count;
};

// the whole patch arrays of `pids`, concatenated on the host in pid order,
// as copies merged where consecutive pids sit next to each other in their
// level's pool; throws on an inactive pid before anything is copied
std::vector<CopyRun> copy_runs(const amr_hierarchy* h, const int* pids, int npatch) {
  std::vector<CopyRun> runs;
  long long pos = 0;
  for (int i = 0; i < npatch; ++i) {
    int64_t off;
    if (amr_patch_offset(h, pids[i], &off) != AMR_OK) throw ArgError("inactive pid");
    const long long cnt = h->dm.lv[h->forest.level[pids[i]]].stride;
    if (!runs.empty() && runs.back().dev + runs.back().count == off)
      runs.back().count += cnt;
    else
      runs.push_back({off, pos, cnt});
    pos += cnt;
  }
  return runs;
}


void validate_config(const amr_config& c) {
  if (c.dim < 1 || c.dim > 3) throw ArgError("dim must be 1, 2 or 3");
  if (c.max_levels < 1 || c.max_levels > AMR_MAX_LEVELS) throw ArgError("bad max_levels");
  if (c.base_cells <= 0) throw ArgError("bad base_cells");
  if (!(c.hi > c.lo)) throw ArgError("empty domain");
  if (!(c.gamma > 1.0)) throw ArgError("gamma must exceed 1");
  if (!(c.cfl > 0.0)) throw ArgError("cfl must be positive");
  // the stage kernel forms 1/(den_L den_R) of the two WENO sides at an edge,
  // products of (eps + beta)^2 terms that must stay normal numbers
  if (!(c.weno_eps >= 1e-20 && c.weno_eps <= 1.0)) throw ArgError("weno_eps must be in [1e-20, 1]");
  if (c.tag_buffer < 0 || c.tag_buffer > 3) throw ArgError("tag_buffer must be in 0..3");
  if (c.scheme != AMR_SCHEME_WENO && c.scheme != AMR_SCHEME_CENTRAL && c.scheme != AMR_SCHEME_CHAR)
    throw ArgError("scheme must be AMR_SCHEME_WENO, _CENTRAL or _CHAR");
  if (c.max_patches <= 0) throw ArgError("max_patches must be positive");
  for (int l = 0; l < c.max_levels; ++l) {
    const int n = c.patch_cells[l];
    if (n < 4 || n % 2) throw ArgError("patch edge must be even and >= 4");
    // in-patch offsets are 32-bit, formed with 24-bit multiplies
    if (n > (c.dim == 3 ? 1024 : (c.dim == 2 ? 16384 : (1 << 22))))
      throw ArgError("patch edge too large (3D 1024, 2D 16384)");
    if (((long long)c.base_cells << l) % n) throw ArgError("level cells not divisible by patch");
    if (l + 1 < c.max_levels && (2 * n) % c.patch_cells[l + 1])
      throw ArgError("fine patch edge must divide twice the coarse edge");
  }
  for (int j = 0; j < c.dim; ++j)
    if (c.periodic[j] != 0 && c.periodic[j] != 1) throw ArgError("periodic flags are 0 or 1");
  if (Kernels::default_variant(c.dim, c.patch_cells, c.max_levels) < 0)
    throw ArgError("patch edges must be multiples of 8 (1D, 2D) or 4 (3D)");
}

void build_devmesh(amr_hierarchy* h) {
  const amr_config& c = h->cfg;
  amr::DevMesh& m = h->dm;
  amr::Forest& f = h->forest;
  m.dim = c.dim;
  m.nvar = c.dim + 2;
  m.nlev = c.max_levels;
  m.scheme = c.scheme;
  m.tile = Kernels::default_variant(c.dim, c.patch_cells, c.max_levels);
  for (int j = 0; j < 3; ++j) m.periodic[j] = j < c.dim ? c.periodic[j] : 1;
  m.max_patches = c.max_patches;
  m.maxc = f.maxc;
  m.gamma = c.gamma;
  m.gm1 = c.gamma - 1.0;
  m.igm1 = 1.0 / m.gm1;
  m.eps = c.weno_eps;
  m.theta = c.tag_theta;
  m.cfl = c.cfl;
  m.tag_buffer = c.tag_buffer;
  // Every box row is a multiple of 8 doubles (64 B) when n is, and a
  // patch's interior starts kNG = 4 doubles into its box rows; a head pad of
  // 4 mod 8 doubles before the first pool puts every interior row on a 64-byte
  // boundary (one memory sector for an 8-wide row instead of two).  The pad is
  // a multiple of nvar, so a box's state offset divided by nvar (its offset
  // in a per-variable plane, and in the cell-tag layout) stays exact.
  long long pad = m.nvar;
  while (pad % 8 != 4) pad += m.nvar;
  long long pool = pad, frp = 0, tg = pad / m.nvar;
  for (int l = 0; l < c.max_levels; ++l) {
    amr::LevelC& L = m.lv[l];
    L.n = f.n[l];
    L.full = L.n + 2 * amr::kNG;
    L.np = f.np[l];
    L.cells = c.base_cells << l;
    L.pid_base = f.pid_base[l];
    L.cap = f.cap[l];
    L.map_off = f.map_off[l];
    L.ratio = f.ratio[l];
    const long long box = ipow(L.full, c.dim);
    L.pool_off = pool;
    L.stride = box * m.nvar;
    L.fr_off = frp;
    L.fr_stride = 2LL * c.dim * m.nvar * ipow(L.n, c.dim - 1);
    L.tag_off = tg;
    L.h = (c.hi - c.lo) / (double)L.cells;
    L.inv_h = 1.0 / L.h;
    pool += L.stride * L.cap;
    frp += L.fr_stride * L.cap;
    tg += box * L.cap;
  }
  h->state_doubles = pool;
  h->fr_doubles = frp;
  h->tag_bytes = tg;
}

// Rebuild work lists on the host and upload them (plus the changed table
// entries) to the device.
// byte offset of the pinned flag slot in h_req (after 2 max_patches bytes of
// requests, 64-byte aligned)
size_t req_flag_offset(int mp) { return ((2 * (size_t)mp + 63) / 64) * 64; }

void sync_tables(amr_hierarchy* h, bool full) {
  ++h->mesh_version;  // recorded step graphs resize their launches before the next replay
  amr::Forest& f = h->forest;
  const int mp = f.max_patches;
  // table deltas
  std::vector<int> pairs;
  auto push_pid = [&](int pid) {
    pairs.push_back((int)(h->off_level + pid));
    pairs.push_back(f.level[pid]);
    pairs.push_back((int)(h->off_parent + pid));
    pairs.push_back(f.parent[pid]);
    pairs.push_back((int)(h->off_nchild + pid));
    pairs.push_back(f.nchild[pid]);
    for (int j = 0; j < 3; ++j) {
      pairs.push_back((int)(h->off_coord + 3LL * pid + j));
      pairs.push_back(f.coord[3 * pid + j]);
    }
    for (int k = 0; k < f.maxc; ++k) {
      pairs.push_back((int)(h->off_child + (long long)pid * f.maxc + k));
      pairs.push_back(f.child[(size_t)pid * f.maxc + k]);
    }
  };
  if (full) {
    std::vector<int> tab(h->tab_ints);
    std::copy(f.level.begin(), f.level.end(), tab.begin() + h->off_level);
    std::copy(f.parent.begin(), f.parent.end(), tab.begin() + h->off_parent);
    std::copy(f.nchild.begin(), f.nchild.end(), tab.begin() + h->off_nchild);
    std::copy(f.coord.begin(), f.coord.end(), tab.begin() + h->off_coord);
    std::copy(f.child.begin(), f.child.end(), tab.begin() + h->off_child);
    std::copy(f.map.begin(), f.map.end(), tab.begin() + h->off_map);
    HIP_OK(hipMemcpyAsync(h->d_tab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice,
                          h->stream));
    h->sync();
  } else {
    std::vector<uint8_t> dirty(mp, 0);
    for (int mi : f.map_dirty) {
      pairs.push_back((int)(h->off_map + mi));
      pairs.push_back(f.map[mi]);
    }
    for (int q : f.touched) dirty[q] = 1;
    for (int pid = 0; pid < mp; ++pid)
      if (dirty[pid]) push_pid(pid);
  }
  f.map_dirty.clear();
  f.touched.clear();

  // active/leaf flags
  h->h_active_leaf.assign(mp, 0);
  for (int pid = 0; pid < mp; ++pid)
    if (f.active[pid]) h->h_active_leaf[pid] = f.nchild[pid] ? 2 : 1;

  // work lists
  std::vector<int>& L = h->lists;
  L.clear();
  const std::vector<int> order = f.sorted_active();
  auto begin_list = [&]() { return (int)L.size(); };
  int a0 = begin_list();
  for (int pid : order) L.push_back(pid);
  const int a1 = begin_list();
  for (int pid : order)
    if (f.is_leaf(pid)) L.push_back(pid);
  // (leaf, ghost region) pairs whose ghost cells have no same-level source:
  // the region's neighbour offset, with components that leave the domain
  // through a non-periodic boundary set to 0 (those ghosts copy the nearest
  // interior cell), points at a missing same-level patch
  const int c0 = begin_list();
  // a leaf whose parent's Moore neighbours all have children has every
  // same-level neighbour (children come in complete sets): nothing to check
  std::vector<int8_t>& pint = h->parent_interior;
  pint.assign(mp, -1);
  auto parent_interior = [&](int P) {
    if (pint[P] < 0) {
      const int lp = f.level[P];
      const int cp[3] = {f.coord[3 * P], f.coord[3 * P + 1], f.coord[3 * P + 2]};
      int8_t ok = 1;
      for (const auto& off : f.moore()) {
        const int q = f.neighbour(lp, cp, off[0], off[1], off[2]);
        if (q == -1 || (q >= 0 && f.is_leaf(q))) {
          ok = 0;
          break;
        }
      }
      pint[P] = ok;
    }
    return pint[P] == 1;
  };
  // A leaf's same-level neighbour at offset src exists iff it is a sibling or
  // the parent's Moore neighbour in that direction has children: children
  // come in complete sets, and by R2 the parent has every Moore neighbour.
  // So one mask per parent (bit = offset code of a neighbour with children)
  // replaces the leaves' own neighbour lookups.  The parents' flags are set
  // first; the leaves are then independent and, on large meshes, split over
  // host threads whose parts are joined in order (the same list).
  std::vector<int>& pkids = h->parent_kids;
  pkids.assign(mp, -1);
  for (int P : order) {
    if (f.is_leaf(P)) continue;
    parent_interior(P);
    const int lp = f.level[P];
    const int cp[3] = {f.coord[3 * P], f.coord[3 * P + 1], f.coord[3 * P + 2]};
    int bits = 0;
    for (const auto& off : f.moore()) {
      const int q = f.neighbour(lp, cp, off[0], off[1], off[2]);
      if (q >= 0 && !f.is_leaf(q)) bits |= 1 << ((off[0] + 1) + 3 * (off[1] + 1) + 9 * (off[2] + 1));
    }
    pkids[P] = bits;
  }
  auto regions = [&](size_t lo, size_t hi, std::vector<int>& out) {
    for (size_t i = lo; i < hi; ++i) {
      const int pid = order[i];
      if (!f.is_leaf(pid) || f.level[pid] == 0) continue;
      const int P = f.parent[pid];
      if (pint[P] == 1) continue;
      const int l = f.level[pid];
      const int r = 2 * f.n[l - 1] / f.n[l];  // children per dimension
      const int c[3] = {f.coord[3 * pid], f.coord[3 * pid + 1], f.coord[3 * pid + 2]};
      const int cpos[3] = {c[0] - f.coord[3 * P] * r, c[1] - f.coord[3 * P + 1] * r,
                           c[2] - f.coord[3 * P + 2] * r};
      const int kids = pkids[P];
      for (const auto& off : f.moore()) {
        int src[3] = {off[0], off[1], off[2]};
        bool self = true;
        int dcode = 0, mul = 1;
        for (int j = 0; j < f.dim; ++j) {
          const int v = c[j] + src[j];
          if ((v < 0 || v >= f.np[l]) && !f.periodic[j]) src[j] = 0;
          self &= src[j] == 0;
          const int w = cpos[j] + src[j];
          dcode += ((w < 0) ? 0 : (w >= r ? 2 : 1)) * mul;
          mul *= 3;
        }
        if (f.dim < 3) dcode += (f.dim == 1 ? 12 : 9);  // centre index of the unused dimensions
        if (self || dcode == 13 || ((kids >> dcode) & 1)) continue;
        out.push_back(pid);
        out.push_back((off[0] + 1) + 3 * (off[1] + 1) + 9 * (off[2] + 1));
      }
    }
  };
  {
    const size_t na = order.size();
    unsigned nth = std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
    if (na < 16384) nth = 1;
    if (nth == 1) {
      regions(0, na, L);
    } else {
      std::vector<std::vector<int>> parts(nth);
      std::vector<std::thread> pool;
      for (unsigned t = 0; t < nth; ++t)
        pool.emplace_back(regions, na * t / nth, na * (t + 1) / nth, std::ref(parts[t]));
      for (auto& th : pool) th.join();
      for (const auto& part : parts) L.insert(L.end(), part.begin(), part.end());
    }
  }
  // the face regions among them (one nonzero offset component)
  const int cf1 = begin_list();
  for (int i = c0; i < cf1; i += 2) {
    const int code = L[i + 1];
    const int nz = (code % 3 != 1) + ((code / 3) % 3 != 1) + ((code / 9) % 3 != 1);
    if (nz == 1) {
      L.push_back(L[i]);
      L.push_back(code);
    }
  }
  // coarsening candidates: patches whose children are all leaves
  const int k0 = begin_list();
  for (int pid : order) {
    if (f.is_leaf(pid)) continue;
    bool all_leaves = true;
    for (int k = 0; k < f.nchild[pid]; ++k) all_leaves &= f.is_leaf(f.child[(size_t)pid * f.maxc + k]);
    if (all_leaves) L.push_back(pid);
  }
  // (leaf, tile) items in brick order (see Forest::leaves_brick_order); the
  // stage kernel's results do not depend on the item order
  const int t0 = begin_list();
  h->leaf_cells = 0;
  for (int pid : f.leaves_brick_order()) {
    h->leaf_cells += ipow(f.n[f.level[pid]], f.dim);
    const int nt = Kernels::tiles_per_patch(h->dm.tile, f.n[f.level[pid]]);
    for (int t = 0; t < nt; ++t) {
      L.push_back(pid);
      L.push_back(t);
    }
  }
  const int r0 = begin_list();
  int nref = 0;
  for (int pid : order) {
    if (!f.is_leaf(pid) || f.level[pid] + 1 >= f.nlev) continue;
    const int l = f.level[pid];
    const int c[3] = {f.coord[3 * pid], f.coord[3 * pid + 1], f.coord[3 * pid + 2]};
    int mask = 0;
    for (int j = 0; j < f.dim; ++j)
      for (int side = 0; side < 2; ++side) {
        const int o = side ? 1 : -1;
        const int qp = f.neighbour(l, c, j == 0 ? o : 0, j == 1 ? o : 0, j == 2 ? o : 0);
        if (qp >= 0 && !f.is_leaf(qp)) mask |= 1 << (2 * j + side);
      }
    if (mask) {
      L.push_back(pid);
      L.push_back(mask);
      ++nref;
    }
  }
  // level-(L-2) patches with children, and level-(L-2) leaves (L-2 >= 1)
  // without coarse/fine faces
  const int lup = f.nlev - 2;
  const int pp0 = begin_list();
  for (int pid : order)
    if (lup >= 0 && f.level[pid] == lup && !f.is_leaf(pid)) L.push_back(pid);
  const int ps0 = begin_list();
  {
    std::vector<uint8_t> has_reflux(f.max_patches, 0);
    for (int i = r0; i < r0 + 2 * nref; i += 2) has_reflux[L[i]] = 1;
    for (int pid : order)
      if (lup >= 1 && f.level[pid] == lup && f.is_leaf(pid) && !has_reflux[pid]) L.push_back(pid);
  }
  const int ps1 = begin_list();
  int rs[amr::kMaxLev + 1] = {};
  for (int l = 0; l < f.nlev; ++l) {
    rs[l] = begin_list();
    if (l == 0) continue;
    for (int pid : order)
      if (f.level[pid] == l) L.push_back(pid);
  }
  rs[f.nlev] = begin_list();
  int ns[amr::kMaxLev + 1] = {};
  for (int l = 0; l < f.nlev; ++l) {
    ns[l] = begin_list();
    for (int q : h->last_created)
      if (f.level[q] == l) L.push_back(q);
  }
  ns[f.nlev] = begin_list();
  if ((long long)L.size() > h->lists_cap) throw StateError("work-list buffer too small");
  const long long np = (long long)pairs.size() / 2;
  if (np > h->pairs_cap) throw StateError("table update buffer too small");
  char* st = h->h_stage;
  int* sl = (int*)st;
  int* sp = sl + h->lists_cap;
  uint8_t* sa = (uint8_t*)(sp + 2 * h->pairs_cap);
  std::copy(L.begin(), L.end(), sl);
  std::copy(pairs.begin(), pairs.end(), sp);
  std::copy(h->h_active_leaf.begin(), h->h_active_leaf.end(), sa);
  if (!L.empty())
    HIP_OK(hipMemcpyAsync(h->d_lists, sl, L.size() * sizeof(int), hipMemcpyHostToDevice,
                          h->stream));
  const int* dd = h->d_dir;
  h->all = {h->d_lists + a0, a1 - a0};
  h->leaves = {h->d_lists + a1, c0 - a1};
  h->cfregions = {h->d_lists + c0, (cf1 - c0) / 2, dd + 2 * kDirCf};
  h->cffaces = {h->d_lists + cf1, (k0 - cf1) / 2, dd + 2 * kDirCfFace};
  h->cands = {h->d_lists + k0, t0 - k0};
  h->tiles = {h->d_lists + t0, (r0 - t0) / 2, dd + 2 * kDirTiles};
  h->reflux = {h->d_lists + r0, nref, dd + 2 * kDirReflux};
  h->post_pairs = {h->d_lists + pp0, ps0 - pp0, dd + 2 * kDirPairs};
  h->post_singles = {h->d_lists + ps0, ps1 - ps0, dd + 2 * kDirSingles};
  for (int l = 0; l < f.nlev; ++l) {
    h->restr[l] = {h->d_lists + rs[l], rs[l + 1] - rs[l], dd + 2 * (kDirRestr + l)};
    h->fresh[l] = {h->d_lists + ns[l], ns[l + 1] - ns[l]};
  }
  {
    // the previous directory upload has completed: every regrid drains the
    // stream before rebuilding the lists
    int* hd = h->h_dir;
    std::fill(hd, hd + 2 * kDirEntries, 0);
    auto put = [&](int e, const amr::ListView& lv) {
      hd[2 * e] = (int)(lv.ptr - h->d_lists);
      hd[2 * e + 1] = lv.count;
    };
    put(kDirCf, h->cfregions);
    put(kDirCfFace, h->cffaces);
    put(kDirTiles, h->tiles);
    put(kDirReflux, h->reflux);
    put(kDirPairs, h->post_pairs);
    put(kDirSingles, h->post_singles);
    for (int l = 0; l < f.nlev; ++l) put(kDirRestr + l, h->restr[l]);
    HIP_OK(hipMemcpyAsync(h->d_dir, hd, 2 * kDirEntries * sizeof(int), hipMemcpyHostToDevice,
                          h->stream));
  }
  HIP_OK(hipMemcpyAsync(h->d_active_leaf, sa, mp, hipMemcpyHostToDevice, h->stream));
  // coarse/fine faces of coarse-side leaves, then the faces whose flux
  // registers refluxing reads: those coarse faces, and every face of a leaf
  // across which no same-level patch lies inside the domain (a fine-side
  // face of a coarse/fine interface, by R2); the stage kernel writes only
  // these registers
  uint8_t* sm = sa + mp;
  std::fill(sm, sm + 2 * mp, (uint8_t)0);
  for (int i = 0; i < nref; ++i) sm[L[r0 + 2 * i]] = (uint8_t)L[r0 + 2 * i + 1];
  uint8_t* sw = sm + mp;
  for (int pid : order)
    if (f.is_leaf(pid)) sw[pid] = sm[pid];
  // a face of a leaf across which no same-level patch lies inside the domain
  // is exactly a face region of the prolonged-ghost list
  for (int i = cf1; i < k0; i += 2) {
    const int code = L[i + 1];
    const int o[3] = {code % 3 - 1, (code / 3) % 3 - 1, (code / 9) % 3 - 1};
    for (int j = 0; j < f.dim; ++j)
      if (o[j] != 0) sw[L[i]] |= (uint8_t)(1 << (2 * j + (o[j] > 0 ? 1 : 0)));
  }
  HIP_OK(hipMemcpyAsync(h->d_cfmask, sm, 2 * mp, hipMemcpyHostToDevice, h->stream));
  if (np > 0) {
    HIP_OK(hipMemcpyAsync(h->d_pairs, sp, pairs.size() * sizeof(int), hipMemcpyHostToDevice,
                          h->stream));
    Kernels::scatter_int(h->d_tab, h->d_pairs, (int)np, h->stream);
    h->check_launch();
  }
}

// Per-patch mode launches one kernel per list entry (the unfused baseline).
template <typename F>
void over_list(amr_hierarchy* h, const amr::ListView& lv, int stride_ints, F launch) {
  if (h->exec_mode == AMR_EXEC_BATCHED) {
    launch(lv.ptr, lv.count);
  } else {
    for (int i = 0; i < lv.count; ++i) launch(lv.ptr + (long long)i * stride_ints, 1);
  }
  h->check_launch();
}

// Grid size (in work items) of a batched launch over a directory list: the
// live count, or while a step graph is recorded at least 1, so that the
// launch node exists and a later regrid can size it (blocks past the live
// count exit at once).
int grid_count(const amr_hierarchy* h, const amr::ListView& lv) {
  return h->capturing ? std::max(lv.count, 1) : lv.count;
}

enum { kGnFill = 0, kGnStage = 1, kGnPost = 2, kGnRestrict = 3 };

int dir_entry(const amr_hierarchy* h, const int* dir) { return (int)(dir - h->d_dir) / 2; }

// Blocks of a launch of this kind over `items` work items (the launchers'
// own grids; at least one block).
int node_grid(const amr_hierarchy* h, int kind, int items) {
  items = std::max(items, 1);
  switch (kind) {
    case kGnFill: return Kernels::fill_cf_grid(h->dm, items);
    case kGnStage: return Kernels::stage_grid(items);
    default: return items;
  }
}

// While a step graph is recorded: the kernel node the last launch added, and
// the directory entries whose live counts size it.
void note_node(amr_hierarchy* h, int kind, int e0, int e1 = -1, int e2 = -1) {
  if (!h->capturing) return;
  hipStreamCaptureStatus st;
  const hipGraphNode_t* deps = nullptr;
  size_t nd = 0;
  HIP_OK(hipStreamGetCaptureInfo_v2(h->stream, &st, nullptr, nullptr, &deps, &nd));
  if (st != hipStreamCaptureStatusActive || nd != 1)
    throw HipError("step capture: expected one open node after a launch");
  amr_hierarchy::GridNode g{};
  g.node = deps[0];
  g.kind = kind;
  g.e[0] = e0;
  g.e[1] = e1;
  g.e[2] = e2;
  g.ne = e2 >= 0 ? 3 : (e1 >= 0 ? 2 : 1);
  int items = 0;
  for (int k = 0; k < g.ne; ++k) items += h->h_dir[2 * g.e[k] + 1];
  g.grid = node_grid(h, kind, items);
  h->gnodes[h->cap_slot].push_back(g);
}

// The step's kernels: in batched mode one launch that reads the list and its
// live count from the list directory (launch(list buffer, grid count,
// directory entry)); per-patch mode as over_list.
template <typename F>
void over_list_dir(amr_hierarchy* h, const amr::ListView& lv, int stride_ints, int kind,
                   F launch) {
  if (h->exec_mode == AMR_EXEC_BATCHED) {
    launch(h->d_lists, grid_count(h, lv), lv.dir);
    h->check_launch();
    note_node(h, kind, dir_entry(h, lv.dir));
    return;
  } else {
    for (int i = 0; i < lv.count; ++i)
      launch(lv.ptr + (long long)i * stride_ints, 1, (const int*)nullptr);
  }
  h->check_launch();
}

void do_fill(amr_hierarchy* h, int buf, const amr::ListView& lv, bool coarse_only = false) {
  over_list(h, lv, 1, [&](const int* p, int c) {
    Kernels::fill(h->dm, h->U[buf], p, c, h->d_flags, coarse_only, h->stream);
  });
}

// ghosts the stage kernel reads from memory: all of them, or with the fused
// halo only the prolonged ones of the face regions (its stencils are
// one-directional; edge and corner regions are read by no stencil)
void stage_fill(amr_hierarchy* h, int buf) {
  if (h->fuse_halo) {
    over_list_dir(h, h->cffaces, 2, kGnFill, [&](const int* p, int c, const int* dir) {
      Kernels::fill_cf(h->dm, h->U[buf], p, c, dir, h->d_flags, h->stream);
    });
  } else {
    do_fill(h, buf, h->leaves);
  }
}

void do_restrict(amr_hierarchy* h, int buf) {
  for (int l = h->forest.nlev - 1; l >= 1; --l)
    over_list_dir(h, h->restr[l], 1, kGnRestrict, [&](const int* p, int c, const int* dir) {
      Kernels::restrict_level(h->dm, h->U[buf], p, c, dir, h->stream);
    });
}

// lam_in (stage 1 of a step): dt comes from that rate slot and is written to
// dt_out; lam_next is then the slot to clear, at stage 3 the slot to fill.
void do_stage(amr_hierarchy* h, int stage, const double* dt,
              unsigned long long* lam_next = nullptr,
              const unsigned long long* lam_in = nullptr, double* dt_out = nullptr) {
  static const int src[4] = {0, 0, 1, 2};
  static const int dst[4] = {0, 1, 2, 0};
  static const double w[4] = {0.0, 1.0, 0.25, 2.0 / 3.0};
  const int s = src[stage], d = dst[stage];
  stage_fill(h, s);
  const Kernels::TileVariant tv = Kernels::variant(h->dm.tile);
  const int tcells = tv.tx * tv.ty * tv.tz;
  over_list_dir(h, h->tiles, 2, kGnStage, [&](const int* p, int c, const int* dir) {
    hipEvent_t a = nullptr, b = nullptr;
    if (h->profiling) h->prof_pair(&a, &b, (long long)c * tcells);
    Kernels::stage(h->dm, stage, h->U[s], h->U[0], h->U[d], h->fr, p, c, dir, dt, h->fuse_halo,
                   (stage == 3 || lam_in) ? lam_next : nullptr, h->d_cfmask, h->stream, a, b,
                   lam_in, dt_out);
  });
  if (h->exec_mode == AMR_EXEC_BATCHED) {
    // refluxing and the restriction of the two finest levels share a launch;
    // coarser levels follow, finest first (lists and counts from the list
    // directory: the three post-stage entries are consecutive)
    const int lup = h->forest.nlev - 2;
    Kernels::post(h->dm, stage, h->U[d], h->fr, h->d_lists, grid_count(h, h->reflux), h->d_lists,
                  grid_count(h, h->post_pairs), h->d_lists, grid_count(h, h->post_singles),
                  h->reflux.dir, lup, true, dt, w[stage], stage == 3 ? lam_next : nullptr,
                  h->stream);
    h->check_launch();
    note_node(h, kGnPost, kDirReflux, kDirPairs, kDirSingles);
    for (int l = lup - 1; l >= 1; --l)
      over_list_dir(h, h->restr[l], 1, kGnRestrict, [&](const int* p, int c, const int* dir) {
        Kernels::restrict_level(h->dm, h->U[d], p, c, dir, h->stream);
      });
  } else {
    over_list(h, h->reflux, 2, [&](const int* p, int c) {
      Kernels::reflux(h->dm, stage, h->U[d], h->fr, p, c, dt, w[stage],
                      stage == 3 ? lam_next : nullptr, h->stream);
    });
    do_restrict(h, d);
  }
}

// CFL rate of the leaf cells of buffer `buf` into rate slot `slot`
void do_rate(amr_hierarchy* h, int buf, int slot) {
  Kernels::zero_u64(h->d_lam + slot, h->stream);
  over_list(h, h->leaves, 1, [&](const int* p, int c) {
    Kernels::max_rate(h->dm, h->U[buf], p, c, h->d_lam + slot, h->stream);
  });
  h->check_launch();
}

void do_dt(amr_hierarchy* h, int buf, double* dt) {
  do_rate(h, buf, 2);
  Kernels::dt_from_rate(h->dm, h->d_lam + 2, dt, nullptr, h->stream);
  h->check_launch();
}

// one step: dt from the current rate slot, three stages; stage 3 and its
// flux correction accumulate the rate of the new U^n into the other slot
void do_step(amr_hierarchy* h, double* dt, int cur) {
  if (h->exec_mode == AMR_EXEC_BATCHED) {
    // dt from the rate slot inside the stage-1 launch
    do_stage(h, 1, dt, h->d_lam + (1 - cur), h->d_lam + cur, dt);
  } else {
    Kernels::dt_from_rate(h->dm, h->d_lam + cur, dt, h->d_lam + (1 - cur), h->stream);
    h->check_launch();
    do_stage(h, 1, dt);
  }
  do_stage(h, 2, dt);
  do_stage(h, 3, dt, h->d_lam + (1 - cur));
}

// Tags of every leaf and of every coarsening candidate (on its restricted
// data), then the requests.
void do_tag(amr_hierarchy* h, int buf, uint8_t* refine, uint8_t* coarsen, uint8_t* cells) {
  // ghosts: with the fused halo only the prolonged ones (coarsening
  // candidates have children, hence every same-level neighbour, and need
  // none); else full fills
  const bool fuse = h->fuse_halo;
  if (fuse) {
    over_list_dir(h, h->cfregions, 2, kGnFill, [&](const int* p, int c, const int* dir) {
      Kernels::fill_cf(h->dm, h->U[buf], p, c, dir, h->d_flags, h->stream);
    });
  } else {
    do_fill(h, buf, h->leaves);
    do_fill(h, buf, h->cands);
  }
  over_list(h, h->leaves, 1, [&](const int* p, int c) {
    Kernels::tag(h->dm, h->U[buf], p, c, h->d_has_tag, cells ? h->d_raw : nullptr, fuse,
                 h->stream);
  });
  over_list(h, h->cands, 1, [&](const int* p, int c) {
    Kernels::tag(h->dm, h->U[buf], p, c, h->d_has_tag, nullptr, fuse, h->stream);
  });
  if (cells)
    over_list(h, h->leaves, 1, [&](const int* p, int c) {
      Kernels::cell_tags(h->dm, h->d_raw, p, c, cells, h->stream);
    });
  Kernels::requests(h->dm, h->d_has_tag, h->d_active_leaf, h->forest.max_patches, refine, coarsen,
                    h->stream);
  h->check_launch();
}

int read_flag(amr_hierarchy* h, int idx) {
  // through a pinned slot after the request buffers: an asynchronous copy
  int* v = reinterpret_cast<int*>(h->h_req + req_flag_offset(h->forest.max_patches));
  HIP_OK(hipMemcpyAsync(v, h->d_flags + idx, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  h->sync();
  return *v;
}

void clear_flags(amr_hierarchy* h) {
  HIP_OK(hipMemsetAsync(h->d_flags, 0, 4 * sizeof(int), h->stream));
}

amr_status regrid_impl(amr_hierarchy* h, const uint8_t* refine, const uint8_t* coarsen,
                       int* ncreated, int* ndeleted) {
  std::vector<int> created, deleted;
  try {
    h->forest.regrid(refine, coarsen, created, deleted);
  } catch (const amr::CapacityError& e) {
    h->err = e.what();
    return AMR_E_CAPACITY;
  }
  if (created.empty() && deleted.empty()) {
    // mesh unchanged: tables, step graphs and the CFL rate stay valid
    h->last_created.clear();
    if (ncreated) *ncreated = 0;
    if (ndeleted) *ndeleted = 0;
    return AMR_OK;
  }
  const std::string why = h->forest.validate_change(created);
  if (!why.empty()) {
    h->err = why;
    return AMR_E_MESH;
  }
  h->last_created = created;
  // the recorded step graphs stay valid: their launches read the lists and
  // counts from the list directory that sync_tables rewrites, and the next
  // replay resizes them (the explicit ghost fill of the unfused path is
  // sized by the leaf count)
  if (!h->fuse_halo) h->step_exec_valid = false;
  h->lam_valid = false;
  sync_tables(h, false);
  // a missing prolongation source (impossible on a valid mesh) raises the
  // sticky error flag read by amr_fill_error; no synchronisation here
  for (int l = 1; l < h->forest.nlev; ++l)
    over_list(h, h->fresh[l], 1, [&](const int* p, int c) {
      Kernels::prolong_new(h->dm, h->U[0], p, c, h->d_flags, h->stream);
    });
  if (ncreated) *ncreated = (int)created.size();
  if (ndeleted) *ndeleted = (int)deleted.size();
  return AMR_OK;
}

template <typename F>
amr_status guarded(amr_hierarchy* h, F body) {
  try {
    return body();
  } catch (const ArgError& e) {
    if (h) h->err = e.what();
    return AMR_E_ARG;
  } catch (const HipError& e) {
    if (h) h->err = e.what();
    return AMR_E_HIP;
  } catch (const amr::CapacityError& e) {
    if (h) h->err = e.what();
    return AMR_E_CAPACITY;
  } catch (const amr::MeshError& e) {
    if (h) h->err = e.what();
    return AMR_E_MESH;
  } catch (const StateError& e) {
    if (h) h->err = e.what();
    return AMR_E_STATE;
  } catch (const std::exception& e) {
    if (h) h->err = e.what();
    return AMR_E_ARG;
  }
}

int buf_ok(int buf) { return buf >= 0 && buf < 3; }

}  // namespace

extern "C" {

amr_status amr_create_hierarchy(const amr_config* cfg, const amr_allocator* alloc,
                                void* hip_stream, amr_hierarchy** out) {
  if (!cfg || !out) return AMR_E_ARG;
  *out = nullptr;
  amr_hierarchy* h = new amr_hierarchy();
  const amr_status st = guarded(h, [&]() -> amr_status {
    validate_config(*cfg);
    h->cfg = *cfg;
    h->stream = (hipStream_t)hip_stream;
    HIP_OK(amr::StateIO::noalloc_scratch(&h->noalloc_scratch));
    if (alloc && alloc->alloc && alloc->free) {
      h->alloc = *alloc;
      h->has_alloc = true;
    }
    h->exec_mode = cfg->exec_mode == AMR_EXEC_PER_PATCH ? AMR_EXEC_PER_PATCH : AMR_EXEC_BATCHED;
    try {
      h->forest.init(*cfg);
    } catch (const std::invalid_argument& e) {
      throw ArgError(e.what());
    }
    h->nvar = cfg->dim + 2;
    build_devmesh(h);
    amr::Forest& f = h->forest;
    const long long mp = f.max_patches;
    h->off_level = 0;
    h->off_parent = mp;
    h->off_nchild = 2 * mp;
    h->off_coord = 3 * mp;
    h->off_child = 6 * mp;
    h->off_map = h->off_child + mp * f.maxc;
    h->tab_ints = h->off_map + (long long)f.map.size();
    if (h->tab_ints > 0x7fffffffLL) throw ArgError("patch tables exceed 2^31 entries");
    for (int b = 0; b < 3; ++b) {
      h->U[b] = (double*)h->dev_alloc(h->state_doubles * sizeof(double));
      HIP_OK(hipMemsetAsync(h->U[b], 0, h->state_doubles * sizeof(double), h->stream));
    }
    h->fr = (double*)h->dev_alloc(h->fr_doubles * sizeof(double));
    h->d_tab = (int*)h->dev_alloc(h->tab_ints * sizeof(int));
    h->d_active_leaf = (uint8_t*)h->dev_alloc(mp);
    // per pid: coarse/fine face mask [0, mp), flux-register write mask [mp, 2 mp)
    h->d_cfmask = (uint8_t*)h->dev_alloc(2 * mp);
    h->d_has_tag = (uint8_t*)h->dev_alloc(mp);
    h->d_refine = (uint8_t*)h->dev_alloc(mp);
    h->d_coarsen = (uint8_t*)h->dev_alloc(mp);
    h->d_raw = (uint8_t*)h->dev_alloc(h->tag_bytes);
    h->d_lam = (unsigned long long*)h->dev_alloc(64);
    h->d_dt = (double*)h->dev_alloc(64);
    h->d_flags = (int*)h->dev_alloc(64);
    long long tiles = 0;  // the most tiles any fitting variant can need
    for (int v = 0; v < Kernels::num_variants(); ++v) {
      if (!Kernels::variant_fits(v, cfg->dim, cfg->patch_cells, cfg->max_levels)) continue;
      long long t = 0;
      for (int l = 0; l < f.nlev; ++l) t += (long long)f.cap[l] * Kernels::tiles_per_patch(v, f.n[l]);
      tiles = std::max(tiles, t);
    }
    // all, leaves, coarsening candidates, reflux (2), post-stage pairs and
    // singles, restriction, new patches: 9 per patch; ghost regions and
    // their faces: 2 per region and patch; tiles: 2 per tile
    const long long regions = ipow(3, cfg->dim) - 1;
    h->lists_cap = 2 * tiles + (9 + 2 * regions + 2 * 2 * cfg->dim) * mp + 64;
    h->d_lists = (int*)h->dev_alloc(h->lists_cap * sizeof(int));
    h->d_dir = (int*)h->dev_alloc(2 * kDirEntries * sizeof(int));
    HIP_OK(hipHostMalloc((void**)&h->h_dir, 2 * kDirEntries * sizeof(int), hipHostMallocDefault));
    h->pairs_cap = mp * (6 + f.maxc) + 2 * (long long)f.map.size() + 64;
    h->pairs_cap = std::min<long long>(h->pairs_cap, 64LL << 20);
    h->d_pairs = (int*)h->dev_alloc(h->pairs_cap * 2 * sizeof(int));
    h->h_stage_bytes = (size_t)h->lists_cap * sizeof(int) + (size_t)h->pairs_cap * 2 * sizeof(int) +
                       3 * (size_t)mp + 256;
    HIP_OK(hipHostMalloc((void**)&h->h_stage, h->h_stage_bytes, hipHostMallocDefault));
    HIP_OK(hipHostMalloc((void**)&h->h_req, req_flag_offset(mp) + 64, hipHostMallocDefault));
    HIP_OK(hipMemsetAsync(h->d_has_tag, 0, mp, h->stream));
    HIP_OK(hipMemsetAsync(h->fr, 0, h->fr_doubles * sizeof(double), h->stream));
    amr::DevMesh& m = h->dm;
    m.level = h->d_tab + h->off_level;
    m.parent = h->d_tab + h->off_parent;
    m.nchild = h->d_tab + h->off_nchild;
    m.coord = h->d_tab + h->off_coord;
    m.child = h->d_tab + h->off_child;
    m.map = h->d_tab + h->off_map;
    sync_tables(h, true);
    clear_flags(h);
    h->sync();
    return AMR_OK;
  });
  if (st != AMR_OK) {
    // keep the message reachable through a minimal object
    h->release_all();
    *out = h;
    return st;
  }
  *out = h;
  return AMR_OK;
}

amr_status amr_destroy_hierarchy(amr_hierarchy* h) {
  if (!h) return AMR_E_ARG;
  (void)hipStreamSynchronize(h->stream);
  h->release_all();
  delete h;
  return AMR_OK;
}

const char* amr_last_error(const amr_hierarchy* h) { return h ? h->err.c_str() : "null hierarchy"; }

amr_status amr_num_patches(const amr_hierarchy* h, int* nactive, int* nleaf) {
  if (!h) return AMR_E_ARG;
  if (nactive) *nactive = h->forest.count_active();
  if (nleaf) *nleaf = h->forest.count_leaves();
  return AMR_OK;
}

amr_status amr_patch_doubles(const amr_hierarchy* h, int level, int64_t* n) {
  if (!h || !n || level < 0 || level >= h->cfg.max_levels) return AMR_E_ARG;
  *n = h->dm.lv[level].stride;
  return AMR_OK;
}

amr_status amr_state_doubles(const amr_hierarchy* h, int64_t* n) {
  if (!h || !n) return AMR_E_ARG;
  *n = h->state_doubles;
  return AMR_OK;
}

amr_status amr_patch_offset(const amr_hierarchy* h, int pid, int64_t* off) {
  if (!h || !off || pid < 0 || pid >= h->forest.max_patches || !h->forest.active[pid])
    return AMR_E_ARG;
  const amr::LevelC& L = h->dm.lv[h->forest.level[pid]];
  *off = L.pool_off + (long long)(pid - L.pid_base) * L.stride;
  return AMR_OK;
}

amr_status amr_state_ptr(const amr_hierarchy* h, int buf, double** dev) {
  if (!h || !dev || !buf_ok(buf)) return AMR_E_ARG;
  *dev = h->U[buf];
  return AMR_OK;
}

amr_status amr_get_patch_table(const amr_hierarchy* h, amr_patch_info* out, int cap, int* n) {
  if (!h || !n) return AMR_E_ARG;
  const amr::Forest& f = h->forest;
  const std::vector<int> order = f.sorted_active();
  *n = (int)order.size();
  for (int i = 0; i < (int)order.size() && i < cap && out; ++i) {
    const int pid = order[i];
    amr_patch_info& r = out[i];
    std::memset(&r, 0, sizeof(r));
    r.pid = pid;
    r.level = f.level[pid];
    for (int j = 0; j < 3; ++j) r.coord[j] = f.coord[3 * pid + j];
    r.parent = f.parent[pid];
    r.nchildren = f.nchild[pid];
    int first = -1;
    for (int k = 0; k < f.nchild[pid]; ++k) {
      const int c = f.child[(size_t)pid * f.maxc + k];
      if (first < 0 || c < first) first = c;
    }
    r.first_child = first;
    for (int k = 0; k < 26; ++k) r.nbr[k] = -1;
    int k = 0;
    for (const auto& off : f.moore()) {
      int q[3];
      r.nbr[k++] = f.shifted(r.level, r.coord, off.data(), q) ? f.lookup(r.level, q) : -1;
    }
  }
  return AMR_OK;
}

amr_status amr_set_state(amr_hierarchy* h, int buf, const double* host, const int* pids,
                         int npatch) {
  if (!h || !buf_ok(buf) || (npatch > 0 && (!host || !pids))) return AMR_E_ARG;
  h->lam_valid = false;
  return guarded(h, [&]() -> amr_status {
    const std::vector<CopyRun> runs = copy_runs(h, pids, npatch);
    for (const CopyRun& r : runs)
      HIP_OK(hipMemcpyAsync(h->U[buf] + r.dev, host + r.host, r.count * sizeof(double),
                            hipMemcpyHostToDevice, h->stream));
    h->sync();
    return AMR_OK;
  });
}

amr_status amr_get_state(const amr_hierarchy* hc, int buf, double* host, const int* pids,
                         int npatch) {
  amr_hierarchy* h = const_cast<amr_hierarchy*>(hc);
  if (!h || !buf_ok(buf) || (npatch > 0 && (!host || !pids))) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    const std::vector<CopyRun> runs = copy_runs(h, pids, npatch);
    for (const CopyRun& r : runs)
      HIP_OK(hipMemcpyAsync(host + r.host, h->U[buf] + r.dev, r.count * sizeof(double),
                            hipMemcpyDeviceToHost, h->stream));
    h->sync();
    return AMR_OK;
  });
}

amr_status amr_set_state_prim(amr_hierarchy* h, int buf, const double* prim, const int* pids,
                              int npatch) {
  if (!h || !buf_ok(buf) || (npatch > 0 && (!prim || !pids))) return AMR_E_ARG;
  h->lam_valid = false;
  return guarded(h, [&]() -> amr_status {
    if (npatch == 0) return AMR_OK;
    const int d = h->cfg.dim, nv = h->nvar;
    // source offset of every patch, all pids checked before anything is written
    std::vector<long long> pos(npatch + 1, 0);
    long long largest = 0;
    for (int i = 0; i < npatch; ++i) {
      int64_t off;
      if (amr_patch_offset(h, pids[i], &off) != AMR_OK) throw ArgError("inactive pid");
      const long long cnt = (long long)nv * ipow(h->dm.lv[h->forest.level[pids[i]]].n, d);
      pos[i + 1] = pos[i] + cnt;
      largest = std::max(largest, cnt);
    }
    // batches of whole patches through one device staging buffer
    const long long cap = std::max(largest, std::min<long long>(pos[npatch], kPrimStageDoubles));
    const int max_batch = (int)std::min<long long>(npatch, kPrimStagePatches);
    const size_t bytes = (size_t)cap * sizeof(double) + (size_t)max_batch * (sizeof(long long) + sizeof(int));
    char* stage = (char*)h->dev_alloc(bytes);
    double* d_prim = (double*)stage;
    long long* d_src = (long long*)(stage + (size_t)cap * sizeof(double));
    int* d_pids = (int*)(d_src + max_batch);
    std::vector<long long> src;
    try {
      for (int i = 0; i < npatch;) {
        int j = i;
        while (j < npatch && j - i < max_batch && pos[j + 1] - pos[i] <= cap) ++j;
        src.resize(j - i);
        for (int k = i; k < j; ++k) src[k - i] = pos[k] - pos[i];
        HIP_OK(hipMemcpyAsync(d_prim, prim + pos[i], (pos[j] - pos[i]) * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
        HIP_OK(hipMemcpyAsync(d_src, src.data(), src.size() * sizeof(long long),
                              hipMemcpyHostToDevice, h->stream));
        HIP_OK(hipMemcpyAsync(d_pids, pids + i, (j - i) * sizeof(int), hipMemcpyHostToDevice,
                              h->stream));
        amr::StateIO::set_prim(h->dm, h->U[buf], d_prim, d_src, d_pids, j - i,
                               h->cfg.gamma - 1.0, h->stream);
        h->check_launch();
        h->sync();  // the staging buffer and src are reused by the next batch
        i = j;
      }
    } catch (...) {
      (void)hipStreamSynchronize(h->stream);
      h->dev_free(stage);
      throw;
    }
    h->dev_free(stage);
    return AMR_OK;
  });
}

static_assert(AMR_NOALLOC_SCRATCH_BYTES == amr::StateIO::kScratchBytes,
              "header and library disagree on the no-allocation scratch size");

amr_status amr_set_state_prim_noalloc(amr_hierarchy* h, int buf, const double* prim,
                                      const int* pids, int npatch) {
  if (!h || !buf_ok(buf) || npatch < 0 || (npatch > 0 && (!prim || !pids))) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    if (npatch == 0) return AMR_OK;
    const int d = h->cfg.dim, nv = h->nvar;
    // scratch layout: primitive values, then (256-byte aligned) the source
    // offset of every patch, then the pids; everything is checked before
    // anything is copied
    std::vector<long long> src(npatch);
    long long total = 0;
    for (int i = 0; i < npatch; ++i) {
      int64_t off;
      if (amr_patch_offset(h, pids[i], &off) != AMR_OK) throw ArgError("inactive pid");
      src[i] = total;
      total += (long long)nv * ipow(h->dm.lv[h->forest.level[pids[i]]].n, d);
    }
    const size_t prim_bytes = ((size_t)total * sizeof(double) + 255) & ~(size_t)255;
    const size_t need = prim_bytes + (size_t)npatch * (sizeof(long long) + sizeof(int));
    if (need > amr::StateIO::kScratchBytes)
      throw ArgError("amr_set_state_prim_noalloc: " + std::to_string(need) +
                     " bytes of primitives and patch indices exceed its " +
                     std::to_string(amr::StateIO::kScratchBytes) +
                     "-byte scratch; split the patches over several calls");
    if (!h->noalloc_scratch) throw StateError("no-allocation scratch not resolved");
    char* base = (char*)h->noalloc_scratch;
    double* d_prim = (double*)base;
    long long* d_src = (long long*)(base + prim_bytes);
    int* d_pids = (int*)(d_src + npatch);
    HIP_OK(hipMemcpyAsync(d_prim, prim, (size_t)total * sizeof(double), hipMemcpyHostToDevice,
                          h->stream));
    HIP_OK(hipMemcpyAsync(d_src, src.data(), (size_t)npatch * sizeof(long long),
                          hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(d_pids, pids, (size_t)npatch * sizeof(int), hipMemcpyHostToDevice,
                          h->stream));
    h->lam_valid = false;
    amr::StateIO::set_prim(h->dm, h->U[buf], d_prim, d_src, d_pids, npatch,
                           h->cfg.gamma - 1.0, h->stream);
    h->check_launch();
    h->sync();  // src lives on this host stack; the scratch is the next call's
    return AMR_OK;
  });
}

amr_status amr_fill_ghosts(amr_hierarchy* h, int buf) {
  if (!h || !buf_ok(buf)) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    do_fill(h, buf, h->all);
    return AMR_OK;
  });
}

amr_status amr_rhs(amr_hierarchy* h, int buf, double* rhs_dev) {
  if (!h || !buf_ok(buf) || !rhs_dev) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    stage_fill(h, buf);
    over_list_dir(h, h->tiles, 2, kGnStage, [&](const int* p, int c, const int* dir) {
      Kernels::stage(h->dm, amr::kModeRHS, h->U[buf], h->U[0], rhs_dev, h->fr, p, c, dir, h->d_dt,
                     h->fuse_halo, nullptr, h->d_cfmask, h->stream);
    });
    over_list(h, h->reflux, 2, [&](const int* p, int c) {
      Kernels::reflux(h->dm, amr::kModeRHS, rhs_dev, h->fr, p, c, h->d_dt, 1.0, nullptr, h->stream);
    });
    return AMR_OK;
  });
}

amr_status amr_compute_dt(amr_hierarchy* h, int buf, double* dt_dev) {
  if (!h || !buf_ok(buf) || !dt_dev) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    do_dt(h, buf, dt_dev);
    return AMR_OK;
  });
}

amr_status amr_rk_stage(amr_hierarchy* h, int stage, const double* dt_dev) {
  if (!h || stage < 1 || stage > 3 || !dt_dev) return AMR_E_ARG;
  h->lam_valid = false;
  return guarded(h, [&]() -> amr_status {
    do_stage(h, stage, dt_dev);
    return AMR_OK;
  });
}

amr_status amr_step(amr_hierarchy* h, double* dt_dev) {
  if (!h) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    double* dt = dt_dev ? dt_dev : h->d_dt;
    const int cur = h->lam_cur;
    if (!h->lam_valid) do_rate(h, 0, cur);
    const bool graph = h->use_graph && h->exec_mode == AMR_EXEC_BATCHED && !h->profiling;
    if (!graph) {
      do_step(h, dt, cur);
    } else {
      if (!h->step_exec_valid) {
        h->step_exec_ok[0] = h->step_exec_ok[1] = false;
        h->step_exec_valid = true;
      }
      if (!h->step_exec_ok[cur] || h->step_exec_dt[cur] != dt) {
        if (!h->cap_stream) HIP_OK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        hipStream_t user = h->stream;
        h->stream = h->cap_stream;
        hipGraph_t g = nullptr;
        h->gnodes[cur].clear();
        HIP_OK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        h->capturing = true;
        h->cap_slot = cur;
        try {
          do_step(h, dt, cur);
        } catch (...) {
          h->capturing = false;
          (void)hipStreamEndCapture(h->stream, &g);
          if (g) (void)hipGraphDestroy(g);
          h->stream = user;
          h->gnodes[cur].clear();
          throw;
        }
        h->capturing = false;
        HIP_OK(hipStreamEndCapture(h->stream, &g));
        h->stream = user;
        if (h->step_exec[cur]) HIP_OK(hipGraphExecDestroy(h->step_exec[cur]));
        h->step_exec[cur] = nullptr;
        if (h->step_graph[cur]) HIP_OK(hipGraphDestroy(h->step_graph[cur]));
        // the recorded graph stays alive: its kernel nodes are the handles
        // through which a regrid resizes the instantiated launches
        h->step_graph[cur] = g;
        HIP_OK(hipGraphInstantiate(&h->step_exec[cur], g, nullptr, nullptr, 0));
        h->step_exec_ok[cur] = true;
        h->step_exec_dt[cur] = dt;
        h->rec_version[cur] = h->mesh_version;
        ++h->step_records;
      } else if (h->rec_version[cur] != h->mesh_version) {
        // the lists changed: each list launch gets the grid of its new length
        for (auto& gn : h->gnodes[cur]) {
          int items = 0;
          for (int k = 0; k < gn.ne; ++k) items += h->h_dir[2 * gn.e[k] + 1];
          const int grid = node_grid(h, gn.kind, items);
          if (grid == gn.grid) continue;
          hipKernelNodeParams p{};
          HIP_OK(hipGraphKernelNodeGetParams(gn.node, &p));
          p.gridDim = dim3(grid);
          HIP_OK(hipGraphExecKernelNodeSetParams(h->step_exec[cur], gn.node, &p));
          HIP_OK(hipGraphKernelNodeSetParams(gn.node, &p));
          gn.grid = grid;
        }
        h->rec_version[cur] = h->mesh_version;
      }
      HIP_OK(hipGraphLaunch(h->step_exec[cur], h->stream));
    }
    h->lam_cur = 1 - cur;
    h->lam_valid = true;
    return AMR_OK;
  });
}

amr_status amr_graph_records(const amr_hierarchy* h, int* recorded) {
  if (!h || !recorded) return AMR_E_ARG;
  *recorded = h->step_records;
  return AMR_OK;
}

amr_status amr_set_graph(amr_hierarchy* h, int enable) {
  if (!h) return AMR_E_ARG;
  if (h->use_graph != (enable != 0)) {
    h->use_graph = enable != 0;
    h->step_exec_valid = false;
  }
  return AMR_OK;
}

amr_status amr_tag(amr_hierarchy* h, int buf, uint8_t* refine_req_dev, uint8_t* coarsen_req_dev,
                   uint8_t* cell_tags_dev) {
  if (!h || !buf_ok(buf)) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    do_tag(h, buf, refine_req_dev, coarsen_req_dev, cell_tags_dev);
    return AMR_OK;
  });
}

amr_status amr_regrid(amr_hierarchy* h, const uint8_t* refine_req_host,
                      const uint8_t* coarsen_req_host, int* ncreated, int* ndeleted) {
  if (!h) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    h->sync();
    return regrid_impl(h, refine_req_host, coarsen_req_host, ncreated, ndeleted);
  });
}

amr_status amr_adapt(amr_hierarchy* h, int* ncreated, int* ndeleted) {
  if (!h) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    const int mp = h->forest.max_patches;
    do_tag(h, 0, h->d_refine, h->d_coarsen, nullptr);
    // into pinned memory: asynchronous copies, one wait
    uint8_t* rq = h->h_req;
    uint8_t* cq = h->h_req + mp;
    HIP_OK(hipMemcpyAsync(rq, h->d_refine, mp, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipMemcpyAsync(cq, h->d_coarsen, mp, hipMemcpyDeviceToHost, h->stream));
    h->sync();
    return regrid_impl(h, rq, cq, ncreated, ndeleted);
  });
}

amr_status amr_check(amr_hierarchy* h, int* nonphysical_count) {
  if (!h) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    HIP_OK(hipMemsetAsync(h->d_flags + 1, 0, sizeof(int), h->stream));
    over_list(h, h->leaves, 1, [&](const int* p, int c) {
      Kernels::check(h->dm, h->U[0], p, c, h->d_flags + 1, h->stream);
    });
    const int bad = read_flag(h, 1);
    if (nonphysical_count) *nonphysical_count = bad;
    if (bad) {
      h->err = "non-physical leaf cells (rho <= 0, p <= 0 or NaN)";
      return AMR_E_NONPHYSICAL;
    }
    return AMR_OK;
  });
}

amr_status amr_judge(amr_hierarchy* h, int* uncovered) {
  if (!h || !uncovered) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    do_tag(h, 0, h->d_refine, nullptr, nullptr);
    HIP_OK(hipMemsetAsync(h->d_flags + 2, 0, sizeof(int), h->stream));
    Kernels::count_nonzero(h->d_refine, h->forest.max_patches, h->d_flags + 2, h->stream);
    h->check_launch();
    *uncovered = read_flag(h, 2);
    return AMR_OK;
  });
}

amr_status amr_set_exec_mode(amr_hierarchy* h, int mode) {
  if (!h || (mode != AMR_EXEC_PER_PATCH && mode != AMR_EXEC_BATCHED)) return AMR_E_ARG;
  h->exec_mode = mode;
  h->step_exec_valid = false;
  return AMR_OK;
}

amr_status amr_set_tile_variant(amr_hierarchy* h, int variant) {
  if (!h) return AMR_E_ARG;
  if (!Kernels::variant_fits(variant, h->cfg.dim, h->cfg.patch_cells, h->cfg.max_levels))
    return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    h->sync();
    h->dm.tile = variant;
    h->last_created.clear();
    sync_tables(h, false);  // rebuilds the (pid, tile) list
    h->step_exec_valid = false;
    return AMR_OK;
  });
}

amr_status amr_get_tile_variant(const amr_hierarchy* h, int* variant, int* tx, int* ty, int* tz,
                                int* threads) {
  if (!h || !variant) return AMR_E_ARG;
  const Kernels::TileVariant t = Kernels::variant(h->dm.tile);
  *variant = h->dm.tile;
  if (tx) *tx = t.tx;
  if (ty) *ty = t.ty;
  if (tz) *tz = t.tz;
  if (threads) *threads = t.threads;
  return AMR_OK;
}

amr_status amr_autotune(amr_hierarchy* h, int reps, int* best, float* best_ms) {
  if (!h || reps < 1) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    // time the stage kernel in RHS mode on U^n, writing into stage buffer B
    // (scratch outside a step) and the flux registers
    double* scratch = h->U[2];
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    const int orig = h->dm.tile;
    int win = orig;
    float win_ms = 1e30f;
    for (int v = 0; v < Kernels::num_variants(); ++v) {
      if (!Kernels::variant_fits(v, h->cfg.dim, h->cfg.patch_cells, h->cfg.max_levels)) continue;
      h->dm.tile = v;
      h->last_created.clear();
      sync_tables(h, false);
      // the launch the batched step makes (list and count from the directory)
      Kernels::stage(h->dm, amr::kModeRHS, h->U[0], h->U[0], scratch, h->fr, h->d_lists,
                     h->tiles.count, h->tiles.dir, h->d_dt, h->fuse_halo, nullptr, h->d_cfmask,
                     h->stream);
      HIP_OK(hipEventRecord(e0, h->stream));
      for (int r = 0; r < reps; ++r)
        Kernels::stage(h->dm, amr::kModeRHS, h->U[0], h->U[0], scratch, h->fr, h->d_lists,
                       h->tiles.count, h->tiles.dir, h->d_dt, h->fuse_halo, nullptr,
                       h->d_cfmask, h->stream);
      HIP_OK(hipEventRecord(e1, h->stream));
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      ms /= reps;
      if (ms < win_ms) {
        win_ms = ms;
        win = v;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->dm.tile = win;
    h->last_created.clear();
    sync_tables(h, false);
    h->step_exec_valid = false;
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return AMR_OK;
  });
}

amr_status amr_set_tag_buffer(amr_hierarchy* h, int cells) {
  if (!h) return AMR_E_ARG;
  if (cells < 0 || cells > 3) {
    h->err = "tag_buffer must be in 0..3";
    return AMR_E_ARG;
  }
  h->cfg.tag_buffer = cells;
  h->dm.tag_buffer = cells;
  h->step_exec_valid = false;
  return AMR_OK;
}

amr_status amr_set_fused_halo(amr_hierarchy* h, int enable) {
  if (!h) return AMR_E_ARG;
  h->fuse_halo = enable != 0;
  h->step_exec_valid = false;
  return AMR_OK;
}

amr_status amr_last_created(const amr_hierarchy* h, int* pids, int cap, int* n) {
  if (!h || !n) return AMR_E_ARG;
  *n = (int)h->last_created.size();
  for (int i = 0; i < *n && i < cap && pids; ++i) pids[i] = h->last_created[i];
  return AMR_OK;
}

amr_status amr_fill_error(amr_hierarchy* h, int* flag) {
  if (!h || !flag) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    *flag = read_flag(h, 0);
    HIP_OK(hipMemsetAsync(h->d_flags, 0, sizeof(int), h->stream));
    return AMR_OK;
  });
}

amr_status amr_forest_replay(const amr_config* cfg, const int32_t* req, int nreq,
                             amr_patch_info* out, int cap, int* n) {
  if (!cfg || !n || (nreq > 0 && !req)) return AMR_E_ARG;
  try {
    validate_config(*cfg);
    amr::Forest f;
    f.init(*cfg);
    const int mp = f.max_patches;
    std::vector<uint8_t> rq(mp), cq(mp);
    int i = 0;
    while (i < nreq) {
      const int round = req[6 * i];
      std::fill(rq.begin(), rq.end(), 0);
      std::fill(cq.begin(), cq.end(), 0);
      for (; i < nreq && req[6 * i] == round; ++i) {
        const int32_t* r = req + 6 * i;
        const int l = r[2];
        if (l < 0 || l >= f.nlev) return AMR_E_ARG;
        const int c[3] = {r[3], r[4], r[5]};
        for (int j = 0; j < f.dim; ++j)
          if (c[j] < 0 || c[j] >= f.np[l]) return AMR_E_ARG;
        const int pid = f.lookup(l, c);
        if (pid < 0) continue;
        (r[1] ? cq : rq)[pid] = 1;
      }
      std::vector<int> created, deleted;
      f.regrid(rq.data(), cq.data(), created, deleted);
      // the full check, and the local one the hierarchy runs after a regrid,
      // which must agree with it
      const bool ok_full = f.validate().empty();
      const bool ok_local = f.validate_change(created).empty();
      if (!ok_full || !ok_local) return AMR_E_MESH;
    }
    const std::vector<int> order = f.sorted_active();
    *n = (int)order.size();
    for (int k = 0; k < (int)order.size() && k < cap && out; ++k) {
      const int pid = order[k];
      amr_patch_info& r = out[k];
      std::memset(&r, 0, sizeof(r));
      r.pid = pid;
      r.level = f.level[pid];
      for (int j = 0; j < 3; ++j) r.coord[j] = f.coord[3 * pid + j];
      r.parent = f.parent[pid];
      r.nchildren = f.nchild[pid];
      r.first_child = f.nchild[pid] ? f.child[(size_t)pid * f.maxc] : -1;
      for (int q = 0; q < 26; ++q) r.nbr[q] = -1;
    }
    return AMR_OK;
  } catch (const amr::CapacityError&) {
    return AMR_E_CAPACITY;
  } catch (const std::exception&) {
    return AMR_E_ARG;
  }
}

amr_status amr_velocity_gradient(amr_hierarchy* h, int buf, double* out_dev) {
  if (!h || !buf_ok(buf) || !out_dev) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    do_fill(h, buf, h->leaves);
    const long long plane = h->state_doubles / h->nvar;
    over_list(h, h->leaves, 1, [&](const int* p, int c) {
      amr::Diagnostics::velocity_gradient(h->dm, h->U[buf], p, c, out_dev, plane, h->stream);
    });
    return AMR_OK;
  });
}

amr_status amr_leaf_cells(const amr_hierarchy* h, int64_t* cells) {
  if (!h || !cells) return AMR_E_ARG;
  *cells = h->leaf_cells;
  return AMR_OK;
}

amr_status amr_profile(amr_hierarchy* h, int enable) {
  if (!h) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    h->sync();
    h->profiling = enable != 0;
    h->ev_used = 0;
    h->ev_cells.clear();
    return AMR_OK;
  });
}

amr_status amr_profile_read(amr_hierarchy* h, double* total_ms, int* launches, int64_t* cells) {
  if (!h || !total_ms || !launches || !cells) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    h->sync();
    double ms = 0.0;
    long long c = 0;
    for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
      float e = 0.f;
      HIP_OK(hipEventElapsedTime(&e, h->ev_pool[i], h->ev_pool[i + 1]));
      ms += e;
    }
    for (long long v : h->ev_cells) c += v;
    *total_ms = ms;
    *launches = (int)h->ev_cells.size();
    *cells = c;
    return AMR_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned refinement predictor
// ---------------------------------------------------------------------------
struct amr_cnn {
  amr_hierarchy* h = nullptr;
  amr_cnn_config cfg{};
  amr::CnnNorm norm{};
  int dim = 2, n = 0, max_batch = 0, t = 0, np = 0;
  long long in_elems = 0;   // BF16 values per input tile
  long long out_cells = 0;  // logits per tile
  std::vector<void*> owned;
  float* params = nullptr;   // FP32 master
  float* m = nullptr;
  float* v = nullptr;
  float* grads = nullptr;
  unsigned short* wb = nullptr;  // BF16 copy
  unsigned short* X = nullptr;   // max_batch input tiles
  unsigned short* A1 = nullptr;
  unsigned short* A2 = nullptr;
  float* Z = nullptr;
  float* G = nullptr;
  float* partials = nullptr;
  float* loss_part = nullptr;
  int loss_blocks = 0;
  int* d_pids = nullptr;   // 2D: pids; 3D: tile items
  long long items_cap = 0;
  uint8_t* d_pred = nullptr;
  void* alloc(size_t bytes) {
    void* p = h->dev_alloc(bytes);
    owned.push_back(p);
    return p;
  }
  void gather(int buf, const int* items, int count, unsigned short* x) const {
    if (dim == 2)
      amr::Cnn::gather(h->dm, h->U[buf], items, count, n, norm, x, h->stream);
    else
      amr::Cnn3::gather(h->dm, h->U[buf], items, count, norm, x, h->stream);
  }
  void forward(const unsigned short* x, int count, unsigned short* a1, unsigned short* a2,
               float* z) const {
    if (dim == 2)
      amr::Cnn::forward(count, n, x, wb, params, a1, a2, z, h->stream);
    else
      amr::Cnn3::forward(count, x, wb, params, a1, a2, z, h->stream);
  }
};

extern "C" {

amr_status amr_cnn_create(amr_hierarchy* h, const amr_cnn_config* cfg, amr_cnn** out) {
  if (!h || !cfg || !out) return AMR_E_ARG;
  *out = nullptr;
  return guarded(h, [&]() -> amr_status {
    const int dim = h->cfg.dim;
    if (dim == 1) throw ArgError("the predictor is implemented for 2D and 3D hierarchies");
    if (dim == 2 && (cfg->patch_cells < 8 || cfg->patch_cells > 32 || cfg->patch_cells % 2))
      throw ArgError("predictor patch edge must be even, 8..32");
    if (dim == 3 && cfg->patch_cells != amr::CNN3_TILE)
      throw ArgError("the 3D predictor works on tiles of edge 8 (patch_cells = 8)");
    if (cfg->max_batch < 1 || cfg->max_batch > 4096) throw ArgError("max_batch must be 1..4096");
    const int nch = dim + 2;
    for (int k = 0; k < nch; ++k)
      if (!(cfg->std[k] > 0.f)) throw ArgError("normalisation std must be positive");
    amr_cnn* c = new amr_cnn();
    c->h = h;
    c->cfg = *cfg;
    c->dim = dim;
    c->n = cfg->patch_cells;
    c->max_batch = cfg->max_batch;
    for (int k = 0; k < 5; ++k) {
      c->norm.mean[k] = k < nch ? cfg->mean[k] : 0.f;
      c->norm.istd[k] = k < nch ? 1.0f / cfg->std[k] : 0.f;
    }
    const int n = c->n;
    const long long N = c->max_batch;
    long long a1e, a2e;
    if (dim == 2) {
      c->np = amr::CNN_NPARAM;
      c->in_elems = 4LL * (n + 6) * (n + 6);
      a1e = 16LL * (n + 4) * (n + 4);
      a2e = 16LL * (n + 2) * (n + 2);
      c->out_cells = (long long)n * n;
      c->items_cap = h->forest.max_patches;
    } else {
      c->np = amr::CNN3_NPARAM;
      c->in_elems = (long long)amr::CNN3_CH * amr::CNN3_P0;
      a1e = (long long)amr::CNN3_CH * amr::CNN3_P1;
      a2e = (long long)amr::CNN3_CH * amr::CNN3_P2;
      c->out_cells = amr::CNN3_P3;
      int tiles = 1;
      for (int l = 0; l < h->forest.nlev; ++l) {
        const int e = h->forest.n[l] / amr::CNN3_TILE;
        tiles = std::max(tiles, e * e * e);
      }
      c->items_cap = (long long)h->forest.max_patches * tiles;
    }
    const int np = c->np;
    try {
      c->params = (float*)c->alloc(np * sizeof(float));
      c->m = (float*)c->alloc(np * sizeof(float));
      c->v = (float*)c->alloc(np * sizeof(float));
      c->grads = (float*)c->alloc(np * sizeof(float));
      c->wb = (unsigned short*)c->alloc(np * sizeof(unsigned short));
      c->X = (unsigned short*)c->alloc(N * c->in_elems * sizeof(unsigned short));
      c->A1 = (unsigned short*)c->alloc(N * a1e * sizeof(unsigned short));
      c->A2 = (unsigned short*)c->alloc(N * a2e * sizeof(unsigned short));
      c->Z = (float*)c->alloc(N * c->out_cells * sizeof(float));
      c->G = (float*)c->alloc(N * c->out_cells * sizeof(float));
      c->partials = (float*)c->alloc(N * np * sizeof(float));
      c->loss_blocks = 256;
      c->loss_part = (float*)c->alloc((c->loss_blocks + 1) * sizeof(float));
      c->d_pids = (int*)c->alloc((size_t)c->items_cap * sizeof(int));
      c->d_pred = (uint8_t*)c->alloc(h->forest.max_patches);
      HIP_OK(hipMemsetAsync(c->params, 0, np * sizeof(float), h->stream));
      HIP_OK(hipMemsetAsync(c->m, 0, np * sizeof(float), h->stream));
      HIP_OK(hipMemsetAsync(c->v, 0, np * sizeof(float), h->stream));
      HIP_OK(hipMemsetAsync(c->wb, 0, np * sizeof(unsigned short), h->stream));
      h->sync();
    } catch (...) {
      amr_cnn_destroy(c);
      throw;
    }
    *out = c;
    return AMR_OK;
  });
}

amr_status amr_cnn_destroy(amr_cnn* c) {
  if (!c) return AMR_E_ARG;
  amr_hierarchy* h = c->h;
  (void)hipStreamSynchronize(h->stream);
  for (void* p : c->owned) {
    auto it = std::find(h->owned.begin(), h->owned.end(), p);
    if (it != h->owned.end()) h->owned.erase(it);
    if (h->has_alloc) h->alloc.free(p, h->alloc.ctx);
    else (void)hipFree(p);
  }
  delete c;
  return AMR_OK;
}

amr_status amr_cnn_num_params(const amr_cnn* c, int* n) {
  if (!c || !n) return AMR_E_ARG;
  *n = c->np;
  return AMR_OK;
}

amr_status amr_cnn_set_weights(amr_cnn* c, const float* host, int n) {
  if (!c || !host || n != c->np) return AMR_E_ARG;
  return guarded(c->h, [&]() -> amr_status {
    HIP_OK(hipMemcpyAsync(c->params, host, n * sizeof(float), hipMemcpyHostToDevice, c->h->stream));
    HIP_OK(hipMemsetAsync(c->m, 0, n * sizeof(float), c->h->stream));
    HIP_OK(hipMemsetAsync(c->v, 0, n * sizeof(float), c->h->stream));
    amr::Cnn::to_bf16(c->params, c->np, c->wb, c->h->stream);
    c->h->check_launch();
    c->t = 0;
    c->h->sync();
    return AMR_OK;
  });
}

amr_status amr_cnn_get_weights(amr_cnn* c, float* host, int n) {
  if (!c || !host || n != c->np) return AMR_E_ARG;
  return guarded(c->h, [&]() -> amr_status {
    HIP_OK(hipMemcpyAsync(host, c->params, n * sizeof(float), hipMemcpyDeviceToHost, c->h->stream));
    c->h->sync();
    return AMR_OK;
  });
}

amr_status amr_cnn_gather(amr_cnn* c, int buf, const int* pids_host, int npatch, uint16_t* x_dev) {
  if (!c || !buf_ok(buf) || npatch < 0 || (npatch > 0 && (!pids_host || !x_dev))) return AMR_E_ARG;
  return guarded(c->h, [&]() -> amr_status {
    amr_hierarchy* h = c->h;
    if (npatch > h->forest.max_patches) throw ArgError("too many pids");
    std::vector<int> items(npatch);
    for (int i = 0; i < npatch; ++i) {
      const int p = pids_host[i];
      if (p < 0 || p >= h->forest.max_patches || !h->forest.active[p] ||
          h->forest.n[h->forest.level[p]] != c->n)
        throw ArgError("gather: pid inactive or of another patch size");
      // a 3D patch of edge 8 is the single tile 0
      items[i] = c->dim == 2 ? p : p * amr::CNN3_MAX_TILES;
    }
    do_fill(h, buf, h->leaves);
    if (npatch > 0)
      HIP_OK(hipMemcpyAsync(c->d_pids, items.data(), npatch * sizeof(int), hipMemcpyHostToDevice,
                            h->stream));
    c->gather(buf, c->d_pids, npatch, (unsigned short*)x_dev);
    h->check_launch();
    h->sync();
    return AMR_OK;
  });
}

amr_status amr_cnn_forward(amr_cnn* c, const uint16_t* x_dev, int npatch, float* logits_dev) {
  if (!c || !x_dev || !logits_dev || npatch < 0 || npatch > c->max_batch) return AMR_E_ARG;
  return guarded(c->h, [&]() -> amr_status {
    c->forward((const unsigned short*)x_dev, npatch, nullptr, nullptr, logits_dev);
    c->h->check_launch();
    return AMR_OK;
  });
}

amr_status amr_cnn_train_step(amr_cnn* c, const uint16_t* x_dev, const uint8_t* labels_dev,
                              int npatch, float lr, float* loss_dev, float* grads_dev) {
  if (!c || !x_dev || !labels_dev || !loss_dev || npatch < 1 || npatch > c->max_batch)
    return AMR_E_ARG;
  return guarded(c->h, [&]() -> amr_status {
    hipStream_t s = c->h->stream;
    const unsigned short* X = (const unsigned short*)x_dev;
    c->forward(X, npatch, c->A1, c->A2, c->Z);
    const long long total = (long long)npatch * c->out_cells;
    amr::Cnn::loss(total, c->Z, labels_dev, c->cfg.pos_weight, c->G, c->loss_part,
                   c->loss_blocks, loss_dev, s);
    if (c->dim == 2)
      amr::Cnn::backward(npatch, c->n, X, c->A1, c->A2, c->G, c->wb, c->partials, c->grads, s);
    else
      amr::Cnn3::backward(npatch, X, c->A1, c->A2, c->G, c->wb, c->partials, c->grads, s);
    if (grads_dev)
      HIP_OK(hipMemcpyAsync(grads_dev, c->grads, c->np * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (lr > 0.f) {
      c->t += 1;
      amr::Cnn::adam(c->params, c->grads, c->m, c->v, lr, c->t, c->np, c->wb, s);
    }
    c->h->check_launch();
    return AMR_OK;
  });
}

amr_status amr_cnn_predict(amr_cnn* c, int buf, float tau, uint8_t* refine_req_dev,
                           uint8_t* coarsen_req_dev) {
  if (!c || !buf_ok(buf) || !(tau > 0.f && tau < 1.f)) return AMR_E_ARG;
  return guarded(c->h, [&]() -> amr_status {
    amr_hierarchy* h = c->h;
    hipStream_t s = h->stream;
    const amr::Forest& f = h->forest;
    // 2D: leaves of edge n; 3D: every 8^3 tile of the leaves whose edge is a
    // multiple of 8
    std::vector<int> items;
    for (int pid = 0; pid < f.max_patches; ++pid) {
      if (!f.active[pid] || !f.is_leaf(pid)) continue;
      const int e = f.n[f.level[pid]];
      if (c->dim == 2) {
        if (e == c->n) items.push_back(pid);
      } else if (e % amr::CNN3_TILE == 0) {
        const int nt = e / amr::CNN3_TILE;
        for (int t = 0; t < nt * nt * nt; ++t) items.push_back(pid * amr::CNN3_MAX_TILES + t);
      }
    }
    if ((long long)items.size() > c->items_cap) throw ArgError("predictor item list overflow");
    do_fill(h, buf, h->leaves);
    HIP_OK(hipMemsetAsync(c->d_pred, 0, f.max_patches, s));
    if (!items.empty())
      HIP_OK(hipMemcpyAsync(c->d_pids, items.data(), items.size() * sizeof(int),
                            hipMemcpyHostToDevice, s));
    const float zt = std::log(tau / (1.0f - tau));
    for (size_t b0 = 0; b0 < items.size(); b0 += (size_t)c->max_batch) {
      const int cnt = (int)std::min<size_t>(c->max_batch, items.size() - b0);
      c->gather(buf, c->d_pids + b0, cnt, c->X);
      c->forward(c->X, cnt, nullptr, nullptr, c->Z);
      if (c->dim == 2)
        amr::Cnn::requests(cnt, c->n, c->Z, c->d_pids + b0, zt, c->d_pred, s);
      else
        amr::Cnn3::requests(cnt, c->Z, c->d_pids + b0, zt, c->d_pred, s);
    }
    Kernels::requests(h->dm, c->d_pred, h->d_active_leaf, f.max_patches, refine_req_dev,
                      coarsen_req_dev, s);
    h->check_launch();
    h->sync();  // items (host vector) copied
    return AMR_OK;
  });
}

amr_status amr_cnn_mfma_selftest(amr_hierarchy* h, const uint16_t* a_dev, const uint16_t* b_dev,
                                 float* d_dev) {
  if (!h || !a_dev || !b_dev || !d_dev) return AMR_E_ARG;
  return guarded(h, [&]() -> amr_status {
    amr::Cnn::mfma_selftest((const unsigned short*)a_dev, (const unsigned short*)b_dev, d_dev,
                            h->stream);
    h->check_launch();
    return AMR_OK;
  });
}

}  // extern "C"

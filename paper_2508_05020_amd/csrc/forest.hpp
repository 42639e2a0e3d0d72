// Host-side patch forest of libamr: patch slots, tree links, per-level patch
// maps, and the mesh adaptation procedures of Section 3.3 of the paper
// (rules R1/R2, Algorithm 1 recursive refinement, Algorithm 2 coarsening).
#pragma once

#include <array>
#include <cstdint>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

#include "amr_internal.hpp"

namespace amr {

struct CapacityError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct MeshError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

class Forest {
 public:
  // Sets up level geometry and slot ranges and creates every level-0 patch.
  void init(const amr_config& cfg);

  int dim = 0, nlev = 0, max_patches = 0, maxc = 0, coarsen_rule = 0;
  int periodic[3] = {0, 0, 0};
  int n[kMaxLev] = {}, np[kMaxLev] = {}, ratio[kMaxLev] = {};
  int pid_base[kMaxLev] = {}, cap[kMaxLev] = {}, map_off[kMaxLev] = {};

  // per pid
  std::vector<int> level, parent, nchild, child, coord;
  std::vector<uint8_t> active;
  // all levels' patch maps (pid or -1), x fastest
  std::vector<int> map;
  // map entries and pids whose rows changed since the device copy was last
  // refreshed
  std::vector<int> map_dirty;
  std::vector<int> touched;

  int map_index(int l, const int c[3]) const {
    int idx = c[0];
    if (dim >= 2) idx += np[l] * c[1];
    if (dim >= 3) idx += np[l] * np[l] * c[2];
    return map_off[l] + idx;
  }
  int lookup(int l, const int c[3]) const { return map[map_index(l, c)]; }
  bool is_leaf(int pid) const { return nchild[pid] == 0; }
  int levels_in_use() const;
  int count_active() const;
  int count_leaves() const;

  // Same-level position c + off; false outside a non-periodic domain.
  bool shifted(int l, const int c[3], const int off[3], int out[3]) const;
  // pid of the same-level patch at c + (o0, o1, o2), offsets in {-1, 0, 1}:
  // -1 when absent, -2 outside a non-periodic domain.
  int neighbour(int l, const int c[3], int o0, int o1, int o2) const {
    const int n = np[l];
    const int o[3] = {o0, o1, o2};
    int q[3] = {0, 0, 0};
    for (int j = 0; j < dim; ++j) {
      int v = c[j] + o[j];
      if (v < 0 || v >= n) {
        if (!periodic[j]) return -2;
        v += v < 0 ? n : -n;
      }
      q[j] = v;
    }
    return map[map_index(l, q)];
  }
  // Level l-1 position whose region contains level-l position c.
  void covering(int l, const int c[3], int out[3]) const;
  // Moore offsets, (dz, dy, dx) lexicographic with dx fastest.
  const std::vector<std::array<int, 3>>& moore() const { return moore_; }

  // Algorithm 1.  Appends new pids to `created`; throws CapacityError.
  void refine(int pid, std::vector<int>& created);
  // Algorithm 2 condition (text reading unless coarsen_rule is literal).
  bool coarsening_allowed(int pid) const;
  void delete_children(int pid, std::vector<int>& deleted);

  // Refinement pass then coarsening pass; transactional on CapacityError.
  void regrid(const uint8_t* refine_req, const uint8_t* coarsen_req,
              std::vector<int>& created, std::vector<int>& deleted);

  // Empty string when R1, R2 and the tree links hold.
  std::string validate() const;
  // The same checks restricted to what the last regrid can have changed
  // (its created patches and coarsened parents).
  std::string validate_change(const std::vector<int>& created) const;

  // Active pids sorted by (level, z, y, x).
  std::vector<int> sorted_active() const;
  // Leaves by level, then in Morton order of their positions: consecutive
  // leaves of a level form compact bricks, so stage tiles that run at the
  // same time on one XCD read each other's cells as halos.
  std::vector<int> leaves_brick_order() const;

 private:
  int alloc(int l, const int c[3], int par);
  void release(int pid);
  std::vector<std::set<int>> free_;
  std::vector<int> coarsened_;  // patches whose children the last regrid deleted
  std::vector<std::array<int, 3>> moore_;
};

}  // namespace amr

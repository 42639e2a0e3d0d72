#include <algorithm>
#include <array>
#include <sstream>

#include "forest.hpp"

namespace amr {

void Forest::init(const amr_config& cfg) {
  dim = cfg.dim;
  nlev = cfg.max_levels;
  max_patches = cfg.max_patches;
  coarsen_rule = cfg.coarsen_rule;
  for (int j = 0; j < 3; ++j) periodic[j] = j < dim ? cfg.periodic[j] : 1;
  maxc = 1;
  long long mapsize = 0;
  for (int l = 0; l < nlev; ++l) {
    n[l] = cfg.patch_cells[l];
    np[l] = (cfg.base_cells << l) / n[l];
    ratio[l] = (l + 1 < nlev) ? 2 * n[l] / cfg.patch_cells[l + 1] : 0;
    int c = 1;
    for (int j = 0; j < dim; ++j) c *= ratio[l];
    if (l + 1 < nlev) maxc = std::max(maxc, c);
    map_off[l] = (int)mapsize;
    long long m = 1;
    for (int j = 0; j < dim; ++j) m *= np[l];
    mapsize += m;
  }
  // slot ranges: explicit capacities where given, level 0 exact otherwise;
  // the remaining slots are shared equally by the other finer levels, a
  // level never getting more than its patch count, with what a capped level
  // leaves over shared again among the rest
  long long l0 = 1;
  for (int j = 0; j < dim; ++j) l0 *= np[0];
  long long full[kMaxLev] = {}, c[kMaxLev] = {};
  long long left = max_patches;
  std::vector<int> open;
  for (int l = 0; l < nlev; ++l) {
    full[l] = 1;
    for (int j = 0; j < dim; ++j) full[l] *= np[l];
    if (cfg.level_capacity[l] > 0) c[l] = std::min<long long>(cfg.level_capacity[l], full[l]);
    else if (l == 0) c[l] = l0;
    else {
      open.push_back(l);
      continue;
    }
    left -= c[l];
  }
  while (!open.empty()) {
    const long long share = std::max<long long>(1, left / (long long)open.size());
    std::vector<int> still;
    for (int l : open) {
      if (full[l] <= share) {
        c[l] = full[l];
        left -= c[l];
      } else {
        still.push_back(l);
      }
    }
    if (still.size() == open.size()) {
      for (int l : still) c[l] = share;
      left -= share * (long long)still.size();
      break;
    }
    open.swap(still);
  }
  long long used = 0;
  for (int l = 0; l < nlev; ++l) {
    pid_base[l] = (int)used;
    cap[l] = (int)c[l];
    used += c[l];
  }
  if (used > max_patches) throw std::invalid_argument("level capacities exceed max_patches");
  if (cap[0] < l0) throw std::invalid_argument("max_patches below the level-0 patch count");

  level.assign(max_patches, -1);
  parent.assign(max_patches, -1);
  nchild.assign(max_patches, 0);
  child.assign((size_t)max_patches * maxc, -1);
  coord.assign((size_t)max_patches * 3, 0);
  active.assign(max_patches, 0);
  map.assign(mapsize, -1);
  map_dirty.clear();
  touched.clear();
  free_.assign(nlev, {});
  for (int l = 0; l < nlev; ++l)
    for (int s = 0; s < cap[l]; ++s) free_[l].insert(pid_base[l] + s);

  moore_.clear();
  const int rz = dim >= 3 ? 1 : 0, ry = dim >= 2 ? 1 : 0;
  for (int dz = -rz; dz <= rz; ++dz)
    for (int dy = -ry; dy <= ry; ++dy)
      for (int dx = -1; dx <= 1; ++dx)
        if (dx || dy || dz) moore_.push_back({dx, dy, dz});

  const int m0 = np[0];
  for (int z = 0; z < (dim >= 3 ? m0 : 1); ++z)
    for (int y = 0; y < (dim >= 2 ? m0 : 1); ++y)
      for (int x = 0; x < m0; ++x) {
        const int c[3] = {x, y, z};
        alloc(0, c, -1);
      }
}


bool Forest::shifted(int l, const int c[3], const int off[3], int out[3]) const {
  out[0] = out[1] = out[2] = 0;
  for (int j = 0; j < dim; ++j) {
    int v = c[j] + off[j];
    if (v < 0 || v >= np[l]) {
      if (!periodic[j]) return false;
      v = ((v % np[l]) + np[l]) % np[l];
    }
    out[j] = v;
  }
  return true;
}

void Forest::covering(int l, const int c[3], int out[3]) const {
  out[0] = out[1] = out[2] = 0;
  for (int j = 0; j < dim; ++j) out[j] = (c[j] * n[l] / 2) / n[l - 1];
}

int Forest::alloc(int l, const int c[3], int par) {
  if (free_[l].empty()) return -1;
  const int pid = *free_[l].begin();
  free_[l].erase(free_[l].begin());
  level[pid] = l;
  parent[pid] = par;
  nchild[pid] = 0;
  active[pid] = 1;
  for (int j = 0; j < 3; ++j) coord[3 * pid + j] = c[j];
  const int mi = map_index(l, c);
  map[mi] = pid;
  map_dirty.push_back(mi);
  touched.push_back(pid);
  if (par >= 0) touched.push_back(par);
  return pid;
}

void Forest::release(int pid) {
  const int l = level[pid];
  const int c[3] = {coord[3 * pid], coord[3 * pid + 1], coord[3 * pid + 2]};
  const int mi = map_index(l, c);
  map[mi] = -1;
  map_dirty.push_back(mi);
  touched.push_back(pid);
  if (parent[pid] >= 0) touched.push_back(parent[pid]);
  active[pid] = 0;
  level[pid] = -1;
  parent[pid] = -1;
  nchild[pid] = 0;
  free_[l].insert(pid);
}

// Algorithm 1: a leaf p first makes each absent Moore neighbour q exist by
// refining the level l-1 patch that covers q (recursively), then receives its
// children.  Positions outside a non-periodic domain count as present.
void Forest::refine(int pid, std::vector<int>& created) {
  if (!active[pid]) throw MeshError("refinement of an inactive patch");
  if (!is_leaf(pid)) return;
  const int l = level[pid];
  if (l + 1 >= nlev) throw MeshError("refinement beyond the finest level");
  const int c[3] = {coord[3 * pid], coord[3 * pid + 1], coord[3 * pid + 2]};
  for (const auto& off : moore_) {
    int q[3];
    if (!shifted(l, c, off.data(), q)) continue;
    if (lookup(l, q) >= 0) continue;
    if (l == 0) throw MeshError("missing level-0 patch");
    int r[3];
    covering(l, q, r);
    const int rp = lookup(l - 1, r);
    if (rp < 0) throw MeshError("covering patch of a missing neighbour is absent");
    refine(rp, created);
  }
  const int rr = ratio[l];
  const int rz = dim >= 3 ? rr : 1, ry = dim >= 2 ? rr : 1;
  int k = 0;
  for (int oz = 0; oz < rz; ++oz)
    for (int oy = 0; oy < ry; ++oy)
      for (int ox = 0; ox < rr; ++ox) {
        int cc[3] = {c[0] * rr + ox, dim >= 2 ? c[1] * rr + oy : 0, dim >= 3 ? c[2] * rr + oz : 0};
        const int q = alloc(l + 1, cc, pid);
        if (q < 0) throw CapacityError("patch pool of a level exhausted");
        child[(size_t)pid * maxc + k] = q;
        nchild[pid] = ++k;
        created.push_back(q);
      }
}

// Algorithm 2, text reading: P needs children, all of them leaves, and none
// of them may be a Moore neighbour of a same-level patch that has children.
// The literal rule instead refuses level 0 and any P with a Moore neighbour
// that has children.
bool Forest::coarsening_allowed(int pid) const {
  if (!active[pid] || is_leaf(pid)) return false;
  const int l = level[pid];
  for (int k = 0; k < nchild[pid]; ++k)
    if (!is_leaf(child[(size_t)pid * maxc + k])) return false;
  if (coarsen_rule == AMR_COARSEN_LITERAL) {
    if (l == 0) return false;
    const int c[3] = {coord[3 * pid], coord[3 * pid + 1], coord[3 * pid + 2]};
    for (const auto& off : moore_) {
      int q[3];
      if (!shifted(l, c, off.data(), q)) continue;
      const int qp = lookup(l, q);
      if (qp >= 0 && !is_leaf(qp)) return false;
    }
    return true;
  }
  for (int k = 0; k < nchild[pid]; ++k) {
    const int ch = child[(size_t)pid * maxc + k];
    const int c[3] = {coord[3 * ch], coord[3 * ch + 1], coord[3 * ch + 2]};
    for (const auto& off : moore_) {
      int q[3];
      if (!shifted(l + 1, c, off.data(), q)) continue;
      const int qp = lookup(l + 1, q);
      if (qp < 0 || parent[qp] == pid) continue;
      if (!is_leaf(qp)) return false;
    }
  }
  return true;
}

void Forest::delete_children(int pid, std::vector<int>& deleted) {
  for (int k = 0; k < nchild[pid]; ++k) {
    const int ch = child[(size_t)pid * maxc + k];
    deleted.push_back(ch);
    release(ch);
    child[(size_t)pid * maxc + k] = -1;
  }
  nchild[pid] = 0;
}

static bool order_less(const Forest& f, int a, int b) {
  if (f.level[a] != f.level[b]) return f.level[a] < f.level[b];
  for (int j = 2; j >= 0; --j)
    if (f.coord[3 * a + j] != f.coord[3 * b + j]) return f.coord[3 * a + j] < f.coord[3 * b + j];
  return a < b;
}

void Forest::regrid(const uint8_t* refine_req, const uint8_t* coarsen_req,
                    std::vector<int>& created, std::vector<int>& deleted) {
  std::vector<int> rq, cq;
  for (int pid = 0; pid < max_patches; ++pid) {
    if (!active[pid]) continue;
    if (refine_req && refine_req[pid] && is_leaf(pid) && level[pid] + 1 < nlev) rq.push_back(pid);
    if (coarsen_req && coarsen_req[pid] && !is_leaf(pid)) cq.push_back(pid);
  }
  std::sort(rq.begin(), rq.end(), [&](int a, int b) { return order_less(*this, a, b); });
  try {
    for (int pid : rq)
      if (active[pid] && is_leaf(pid)) refine(pid, created);
  } catch (const CapacityError&) {
    // undo: remove every patch created in this pass, newest first
    for (auto it = created.rbegin(); it != created.rend(); ++it) {
      const int q = *it;
      const int par = parent[q];
      release(q);
      if (par >= 0) {
        nchild[par] = 0;
        for (int k = 0; k < maxc; ++k) child[(size_t)par * maxc + k] = -1;
      }
    }
    created.clear();
    throw;
  }
  std::vector<uint8_t> fresh_parent(max_patches, 0);
  for (int q : created) fresh_parent[parent[q]] = 1;
  std::sort(cq.begin(), cq.end(), [&](int a, int b) {
    if (level[a] != level[b]) return level[a] > level[b];
    return order_less(*this, a, b);
  });
  coarsened_.clear();
  for (int pid : cq) {
    if (!active[pid] || fresh_parent[pid]) continue;
    if (coarsening_allowed(pid)) {
      delete_children(pid, deleted);
      coarsened_.push_back(pid);
    }
  }
}

std::string Forest::validate_change(const std::vector<int>& created) const {
  // R2 can only fail at patches with children near the change: the parents
  // of created patches (and the patches Algorithm 1 refined around them,
  // which are parents of created patches too), and patches one level below a
  // coarsened patch that border its former children.
  auto r2 = [&](int q) -> bool {
    const int l = level[q];
    const int c[3] = {coord[3 * q], coord[3 * q + 1], coord[3 * q + 2]};
    for (const auto& off : moore_)
      if (neighbour(l, c, off[0], off[1], off[2]) == -1) return false;
    return true;
  };
  for (int q : created) {
    const int l = level[q];
    const int c[3] = {coord[3 * q], coord[3 * q + 1], coord[3 * q + 2]};
    if (!active[q] || lookup(l, c) != q) return "patch map disagrees with the patch table";
    int r[3];
    covering(l, c, r);
    if (lookup(l - 1, r) != parent[q]) return "parent link broken";
    if (!r2(parent[q])) return "R2: a refined patch has an absent Moore neighbour";
  }
  for (int p : coarsened_) {
    const int l = level[p] + 1;
    if (l >= nlev) continue;
    // former children's region on level l, grown by one patch
    const int r = ratio[level[p]];
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int j = 0; j < dim; ++j) {
      lo[j] = coord[3 * p + j] * r - 1;
      hi[j] = coord[3 * p + j] * r + r;
    }
    for (int z = lo[2]; z <= (dim >= 3 ? hi[2] : lo[2]); ++z)
      for (int y = lo[1]; y <= (dim >= 2 ? hi[1] : lo[1]); ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) {
          int q3[3] = {x, y, z};
          bool in = true;
          for (int j = 0; j < dim; ++j) {
            int& v = q3[j];
            if (v < 0 || v >= np[l]) {
              if (!periodic[j]) in = false;
              else v = (v % np[l] + np[l]) % np[l];
            }
          }
          if (!in) continue;
          const int q = lookup(l, q3);
          if (q >= 0 && !is_leaf(q) && !r2(q))
            return "R2: a patch with children borders a coarsened region";
        }
  }
  return "";
}

std::string Forest::validate() const {
  std::ostringstream why;
  const int m0 = np[0];
  for (int z = 0; z < (dim >= 3 ? m0 : 1); ++z)
    for (int y = 0; y < (dim >= 2 ? m0 : 1); ++y)
      for (int x = 0; x < m0; ++x) {
        const int c[3] = {x, y, z};
        if (lookup(0, c) < 0) return "R1: a level-0 patch is missing";
      }
  for (int pid = 0; pid < max_patches; ++pid) {
    if (!active[pid]) continue;
    const int l = level[pid];
    const int c[3] = {coord[3 * pid], coord[3 * pid + 1], coord[3 * pid + 2]};
    if (lookup(l, c) != pid) return "patch map disagrees with the patch table";
    if (l > 0) {
      int r[3];
      covering(l, c, r);
      if (lookup(l - 1, r) != parent[pid]) return "parent link broken";
    }
    if (nchild[pid]) {
      for (const auto& off : moore_) {
        int q[3];
        if (!shifted(l, c, off.data(), q)) continue;
        if (lookup(l, q) < 0) {
          why << "R2: patch " << pid << " has children but a Moore neighbour is absent";
          return why.str();
        }
      }
    }
  }
  return "";
}

int Forest::levels_in_use() const {
  int m = 0;
  for (int pid = 0; pid < max_patches; ++pid)
    if (active[pid]) m = std::max(m, level[pid] + 1);
  return m;
}

int Forest::count_active() const {
  int c = 0;
  for (int pid = 0; pid < max_patches; ++pid) c += active[pid] ? 1 : 0;
  return c;
}

int Forest::count_leaves() const {
  int c = 0;
  for (int pid = 0; pid < max_patches; ++pid) c += (active[pid] && nchild[pid] == 0) ? 1 : 0;
  return c;
}

std::vector<int> Forest::sorted_active() const {
  std::vector<int> out;
  // small level maps: their index order is (z, y, x) within a level, so a
  // scan of the maps level by level yields the order without sorting
  if (map.size() <= 4 * (size_t)max_patches) {
    for (int l = 0; l < nlev; ++l) {
      size_t cells = 1;
      for (int j = 0; j < dim; ++j) cells *= (size_t)np[l];
      const int* m = map.data() + map_off[l];
      for (size_t i = 0; i < cells; ++i)
        if (m[i] >= 0) out.push_back(m[i]);
    }
    return out;
  }
  // (level, z, y, x, pid) packed into one 64-bit key when the fields fit,
  // each field as wide as this forest needs, else the comparator
  auto width = [](long long v) {  // bits for the values 0 .. v - 1
    int b = 0;
    while (b < 62 && (1LL << b) < v) ++b;
    return b;
  };
  int npmax = 1;
  for (int l = 0; l < nlev; ++l) npmax = std::max(npmax, np[l]);
  const int bp = width(max_patches), bc = width(npmax), bl = width(nlev);
  const int ob = bl + dim * bc;  // ordering bits above the pid field
  if (bp + ob <= 64) {
    std::vector<uint64_t> keys;
    for (int pid = 0; pid < max_patches; ++pid) {
      if (!active[pid]) continue;
      uint64_t k = (uint64_t)level[pid];
      for (int j = dim - 1; j >= 0; --j) k = (k << bc) | (uint64_t)coord[3 * pid + j];
      keys.push_back((k << bp) | (uint64_t)pid);
    }
    if (keys.size() < 4096) {
      std::sort(keys.begin(), keys.end());
    } else {
      // LSD radix sort on the ordering bits, 16-bit digits; the keys are
      // distinct, so the order is the comparison sort's
      std::vector<uint64_t> tmp(keys.size());
      std::vector<uint32_t> cnt(65537);
      for (int sh = bp; sh < bp + ob; sh += 16) {
        std::fill(cnt.begin(), cnt.end(), 0u);
        for (const uint64_t k : keys) ++cnt[((k >> sh) & 0xffffu) + 1];
        for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
        for (const uint64_t k : keys) tmp[cnt[(k >> sh) & 0xffffu]++] = k;
        keys.swap(tmp);
      }
    }
    out.reserve(keys.size());
    const uint64_t pm = (bp >= 64) ? ~0ull : ((1ull << bp) - 1);
    for (uint64_t k : keys) out.push_back((int)(k & pm));
    return out;
  }
  for (int pid = 0; pid < max_patches; ++pid)
    if (active[pid]) out.push_back(pid);
  std::sort(out.begin(), out.end(), [&](int a, int b) { return order_less(*this, a, b); });
  return out;
}


namespace {
// The low bits of v spread to every second (third) bit position.
uint64_t spread2(uint64_t v) {
  v &= 0xffffffffull;
  v = (v | (v << 16)) & 0x0000ffff0000ffffull;
  v = (v | (v << 8)) & 0x00ff00ff00ff00ffull;
  v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0full;
  v = (v | (v << 2)) & 0x3333333333333333ull;
  return (v | (v << 1)) & 0x5555555555555555ull;
}
uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x001f00000000ffffull;
  v = (v | (v << 16)) & 0x001f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  return (v | (v << 2)) & 0x1249249249249249ull;
}
// Morton code of a patch position: bit b of coordinate j at bit b dim + j
// (x lowest; 13 bits per coordinate).
uint64_t morton(const int* c, int dim) {
  const uint64_t m13 = (1u << 13) - 1;
  if (dim == 1) return (uint64_t)c[0] & m13;
  if (dim == 2) return spread2(c[0] & m13) | (spread2(c[1] & m13) << 1);
  return spread3(c[0] & m13) | (spread3(c[1] & m13) << 1) | (spread3(c[2] & m13) << 2);
}
}  // namespace

std::vector<int> Forest::leaves_brick_order() const {
  // (level, Morton code, pid) packed into one key: level in bits 60..63, the
  // code in bits 21..59 (13 bits per coordinate), the pid in bits 0..20;
  // else the comparator on (level, code, pid)
  std::vector<int> out;
  bool packed = max_patches <= (1 << 21) && nlev <= 16;
  for (int l = 0; l < nlev; ++l) packed &= np[l] <= (1 << 13);
  if (packed) {
    std::vector<uint64_t> keys;
    for (int pid = 0; pid < max_patches; ++pid) {
      if (!active[pid] || nchild[pid]) continue;
      keys.push_back(((uint64_t)level[pid] << 60) | (morton(&coord[3 * pid], dim) << 21) |
                     (uint64_t)pid);
    }
    if (keys.size() < 4096) {
      std::sort(keys.begin(), keys.end());
    } else {
      // LSD radix sort on bits 21..63, 16-bit digits (the keys are distinct)
      std::vector<uint64_t> tmp(keys.size());
      std::vector<uint32_t> cnt(65537);
      for (const int sh : {21, 37, 53}) {
        std::fill(cnt.begin(), cnt.end(), 0u);
        for (const uint64_t k : keys) ++cnt[((k >> sh) & 0xffffu) + 1];
        for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
        for (const uint64_t k : keys) tmp[cnt[(k >> sh) & 0xffffu]++] = k;
        keys.swap(tmp);
      }
    }
    out.reserve(keys.size());
    for (uint64_t k : keys) out.push_back((int)(k & ((1u << 21) - 1)));
    return out;
  }
  for (int pid = 0; pid < max_patches; ++pid)
    if (active[pid] && !nchild[pid]) out.push_back(pid);
  std::sort(out.begin(), out.end(), [&](int a, int b) {
    if (level[a] != level[b]) return level[a] < level[b];
    const uint64_t ma = morton(&coord[3 * a], dim), mb = morton(&coord[3 * b], dim);
    return ma != mb ? ma < mb : a < b;
  });
  return out;
}

}  // namespace amr

// Host forest builder and level tables (see forest.hpp).
#include "forest.hpp"

#include <algorithm>
#include <cstdio>

#include "../../include/lbm_refined.h"

namespace lbm {

uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t key = 0;
  for (int b = 0; b < 21; ++b) {
    key |= uint64_t((x >> b) & 1u) << (3 * b);
    key |= uint64_t((y >> b) & 1u) << (3 * b + 1);
    key |= uint64_t((z >> b) & 1u) << (3 * b + 2);
  }
  return key;
}

static inline int wrap(int v, int d) {
  v %= d;
  return v < 0 ? v + d : v;
}

bool Forest::is_leaf(int level, int x, int y, int z) const {
  return leaves_.count(block_key(level, x, y, z)) != 0;
}

int Forest::covering_level(int level, int x, int y, int z) const {
  x = wrap(x, dims(level, 0));
  y = wrap(y, dims(level, 1));
  z = wrap(z, dims(level, 2));
  for (int l = level; l >= 0; --l) {
    const int s = level - l;
    if (is_leaf(l, x >> s, y >> s, z >> s)) return l;
  }
  return level + 1;
}

void Forest::split(const Leaf& l) {
  leaves_.erase(block_key(l.level, l.x, l.y, l.z));
  for (int o = 0; o < 8; ++o)
    leaves_.insert(block_key(l.level + 1, 2 * l.x + (o & 1), 2 * l.y + ((o >> 1) & 1), 2 * l.z + (o >> 2)));
}

static Leaf unpack(uint64_t k) {
  Leaf l;
  l.level = int(k >> 57);
  l.x = int((k >> 38) & 0x7FFFF);
  l.y = int((k >> 19) & 0x7FFFF);
  l.z = int(k & 0x7FFFF);
  return l;
}

// Ripple balance: visit levels from the finest down; for each leaf of level
// L, every neighbouring position covered by a leaf coarser than L-1 gets
// that leaf split along the way down to level L-1.  Leaves created here are
// coarser than L and are visited when their own level comes.
void Forest::enforce_balance() {
  int lmax = 0;
  for (uint64_t k : leaves_) lmax = std::max(lmax, unpack(k).level);
  for (int L = lmax; L >= 2; --L) {
    std::vector<Leaf> cur;
    for (uint64_t k : leaves_) {
      Leaf l = unpack(k);
      if (l.level == L) cur.push_back(l);
    }
    for (const Leaf& l : cur) {
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            if (!dx && !dy && !dz) continue;
            const int px = wrap(l.x + dx, dims(L, 0)), py = wrap(l.y + dy, dims(L, 1)),
                      pz = wrap(l.z + dz, dims(L, 2));
            for (;;) {
              const int cl = covering_level(L, px, py, pz);
              if (cl >= L - 1) break;
              const int s = L - cl;
              split(Leaf{cl, px >> s, py >> s, pz >> s});
            }
          }
    }
  }
}

bool Forest::balanced() const {
  for (uint64_t k : leaves_) {
    const Leaf l = unpack(k);
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (!dx && !dy && !dz) continue;
          if (covering_level(l.level, l.x + dx, l.y + dy, l.z + dz) < l.level - 1) return false;
        }
  }
  return true;
}

bool Forest::check_cover(std::string& err) const {
  // every leaf inside the grid, and the volumes add up to the domain with no
  // position of the finest level claimed twice
  int lmax = 0;
  for (uint64_t k : leaves_) lmax = std::max(lmax, unpack(k).level);
  if (lmax > 20) {
    err = "level above 20";
    return false;
  }
  // volume in units of level-lmax blocks, exact in 128-bit integers
  unsigned __int128 vol = 0;
  for (uint64_t k : leaves_) {
    const Leaf l = unpack(k);
    if (l.x < 0 || l.y < 0 || l.z < 0 || l.x >= dims(l.level, 0) || l.y >= dims(l.level, 1) ||
        l.z >= dims(l.level, 2)) {
      err = "leaf outside the root grid";
      return false;
    }
    // no ancestor may also be a leaf
    for (int a = l.level - 1; a >= 0; --a) {
      const int s = l.level - a;
      if (is_leaf(a, l.x >> s, l.y >> s, l.z >> s)) {
        err = "overlapping leaves";
        return false;
      }
    }
    vol += (unsigned __int128)1 << (3 * (lmax - l.level));
  }
  const unsigned __int128 domain = ((unsigned __int128)R[0] * R[1] * R[2]) << (3 * lmax);
  if (vol != domain) {
    err = "leaves do not cover the domain";
    return false;
  }
  return true;
}

void Forest::finalize() {
  max_level = 0;
  for (uint64_t k : leaves_) max_level = std::max(max_level, unpack(k).level);
  by_level_.assign(max_level + 1, {});
  for (uint64_t k : leaves_) {
    const Leaf l = unpack(k);
    by_level_[l.level].push_back(l);
  }
  for (auto& v : by_level_)
    std::sort(v.begin(), v.end(), [](const Leaf& a, const Leaf& b) {
      return morton3(a.x, a.y, a.z) < morton3(b.x, b.y, b.z);
    });
}

int Forest::build_from_leaves(const int R_[3], int n_, const int32_t* leaves, int64_t count, bool balance,
                              std::string& err) {
  for (int a = 0; a < 3; ++a) R[a] = R_[a];
  n = n_;
  leaves_.clear();
  for (int64_t i = 0; i < count; ++i) {
    const int32_t* l = leaves + 4 * i;
    if (l[0] < 0 || l[0] > 20) {
      err = "leaf level out of range";
      return LBM_E_INVALID;
    }
    if (!leaves_.insert(block_key(l[0], l[1], l[2], l[3])).second) {
      err = "duplicate leaf";
      return LBM_E_COVER;
    }
  }
  if (!check_cover(err)) return LBM_E_COVER;
  if (!balanced()) {
    if (!balance) {
      err = "leaves violate the 2:1 balance";
      return LBM_E_UNBALANCED;
    }
    enforce_balance();
  }
  finalize();
  return LBM_OK;
}

int Forest::build_from_callback(const int R_[3], int n_, int max_level_, int (*refine)(int, int, int, int, void*),
                                void* user, std::string& err) {
  for (int a = 0; a < 3; ++a) R[a] = R_[a];
  n = n_;
  leaves_.clear();
  std::vector<Leaf> cur;
  for (int z = 0; z < R[2]; ++z)
    for (int y = 0; y < R[1]; ++y)
      for (int x = 0; x < R[0]; ++x) cur.push_back(Leaf{0, x, y, z});
  for (const Leaf& l : cur) leaves_.insert(block_key(0, l.x, l.y, l.z));
  for (int L = 0; L < max_level_ && refine; ++L) {
    std::vector<Leaf> next;
    for (const Leaf& l : cur) {
      if (refine(L, l.x, l.y, l.z, user)) {
        split(l);
        for (int o = 0; o < 8; ++o)
          next.push_back(Leaf{L + 1, 2 * l.x + (o & 1), 2 * l.y + ((o >> 1) & 1), 2 * l.z + (o >> 2)});
      }
    }
    cur.swap(next);
  }
  enforce_balance();
  if (!check_cover(err)) return LBM_E_COVER;
  finalize();
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// level tables
// ---------------------------------------------------------------------------

namespace {

struct SlotMap {
  std::unordered_map<uint64_t, int32_t> real, ghost;
  int32_t find(int L, int x, int y, int z) const {
    const uint64_t k = block_key(L, x, y, z);
    auto it = real.find(k);
    if (it != real.end()) return it->second;
    auto g = ghost.find(k);
    return g == ghost.end() ? kNbrNone : g->second;
  }
};

// Live zones of a ghost block whose real neighbours are given by `real_dir`
// (27 flags, offset index (dx+1) + 3 (dy+1) + 9 (dz+1)).
uint32_t live_zones(const bool real_dir[27]) {
  uint32_t mask = 0;
  for (int zz = 0; zz < 3; ++zz)
    for (int zy = 0; zy < 3; ++zy)
      for (int zx = 0; zx < 3; ++zx) {
        const int zone[3] = {zx, zy, zz};
        bool live = false;
        for (int d = 0; d < 27 && !live; ++d) {
          if (d == kNbrSelf || !real_dir[d]) continue;
          const int off[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
          bool ok = true;
          for (int a = 0; a < 3; ++a) {
            if (off[a] == 0) continue;
            if (off[a] == -1 && zone[a] != 0) ok = false;
            if (off[a] == 1 && zone[a] != 2) ok = false;
          }
          live = ok;
        }
        if (live) mask |= 1u << (zx + 3 * zy + 9 * zz);
      }
  return mask;
}

}  // namespace

int build_level_tables(const Forest& f, std::vector<LevelTables>& out, std::string& err) {
  const int n = f.n;
  const int n3 = n * n * n;
  const int tile = std::min(256, n3);
  const int nlev = f.num_levels();
  out.assign(nlev, LevelTables{});
  std::vector<SlotMap> maps(nlev);

  // pass 1: slots of every level
  for (int L = 0; L < nlev; ++L) {
    LevelTables& t = out[L];
    t.level = L;
    t.n = n;
    t.tile = tile;
    t.tiles_per_block = n3 / tile;
    const auto& leaves = f.level_leaves(L);
    t.nreal = int(leaves.size());
    for (int b = 0; b < t.nreal; ++b) maps[L].real[block_key(L, leaves[b].x, leaves[b].y, leaves[b].z)] = b;
    std::vector<Leaf> ghosts;
    if (L > 0) {
      std::unordered_set<uint64_t> seen;
      for (const Leaf& l : leaves)
        for (int d = 0; d < 27; ++d) {
          if (d == kNbrSelf) continue;
          const int px = wrap(l.x + d % 3 - 1, f.dims(L, 0)), py = wrap(l.y + (d / 3) % 3 - 1, f.dims(L, 1)),
                    pz = wrap(l.z + d / 9 - 1, f.dims(L, 2));
          const int cl = f.covering_level(L, px, py, pz);
          if (cl == L - 1) {
            if (seen.insert(block_key(L, px, py, pz)).second) ghosts.push_back(Leaf{L, px, py, pz});
          } else if (cl < L - 1) {
            err = "2:1 balance violated";
            return LBM_E_UNBALANCED;
          }
        }
    }
    std::sort(ghosts.begin(), ghosts.end(), [](const Leaf& a, const Leaf& b) {
      return morton3(a.x, a.y, a.z) < morton3(b.x, b.y, b.z);
    });
    t.nghost = int(ghosts.size());
    for (int g = 0; g < t.nghost; ++g) {
      maps[L].ghost[block_key(L, ghosts[g].x, ghosts[g].y, ghosts[g].z)] = t.nreal + g;
      t.ghost_pos.push_back(ghosts[g].x);
      t.ghost_pos.push_back(ghosts[g].y);
      t.ghost_pos.push_back(ghosts[g].z);
    }
  }

  // pass 2: neighbour tables, zones, parents, children, work lists
  for (int L = 0; L < nlev; ++L) {
    LevelTables& t = out[L];
    const int nslot = t.nreal + t.nghost;
    t.nbr.assign(size_t(nslot) * 27, kNbrNone);
    t.zmask.assign(nslot, 0);
    t.parent.assign(nslot, -1);
    t.flags.assign(nslot, 0);
    t.child_ghost.assign(size_t(t.nreal) * 8, -1);
    const auto& leaves = f.level_leaves(L);
    for (int s = 0; s < nslot; ++s) {
      const bool real = s < t.nreal;
      int bx, by, bz;
      if (real) {
        bx = leaves[s].x, by = leaves[s].y, bz = leaves[s].z;
      } else {
        const int g = s - t.nreal;
        bx = t.ghost_pos[3 * g], by = t.ghost_pos[3 * g + 1], bz = t.ghost_pos[3 * g + 2];
      }
      bool real_dir[27] = {};
      uint32_t fl = real ? uint32_t(kReal) : 0u;
      bool all_same = true;
      for (int d = 0; d < 27; ++d) {
        const int px = wrap(bx + d % 3 - 1, f.dims(L, 0)), py = wrap(by + (d / 3) % 3 - 1, f.dims(L, 1)),
                  pz = wrap(bz + d / 9 - 1, f.dims(L, 2));
        int32_t v = maps[L].find(L, px, py, pz);
        if (v == kNbrNone && f.covering_level(L, px, py, pz) == L + 1) v = kNbrFine;
        t.nbr[size_t(s) * 27 + d] = v;
        real_dir[d] = v >= 0 && v < t.nreal;
        if (d != kNbrSelf) {
          if (!real_dir[d]) all_same = false;
          if (v == kNbrFine) fl |= kHasFine;
          if (v >= t.nreal) fl |= kHasGhost;
          if (v == kNbrFine && !real) {
            err = "ghost block touches the finer region";
            return LBM_E_UNBALANCED;
          }
        }
      }
      if (real && all_same) fl |= kAllSameLevel;
      t.flags[s] = fl;
      t.zmask[s] = real ? 0x7FFFFFFu : live_zones(real_dir);
      if (!real) {
        const int32_t ps = maps[L - 1].find(L - 1, bx >> 1, by >> 1, bz >> 1);
        if (ps < 0 || ps >= out[L - 1].nreal) {
          err = "ghost block without a parent leaf";
          return LBM_E_UNBALANCED;
        }
        t.parent[s] = ps * 8 + ((bx & 1) | ((by & 1) << 1) | ((bz & 1) << 2));
      } else if (L + 1 < nlev) {
        for (int o = 0; o < 8; ++o) {
          const uint64_t k = block_key(L + 1, 2 * bx + (o & 1), 2 * by + ((o >> 1) & 1), 2 * bz + (o >> 2));
          auto g = maps[L + 1].ghost.find(k);
          if (g != maps[L + 1].ghost.end()) t.child_ghost[size_t(s) * 8 + o] = g->second;
        }
      }
    }

    // work tiles: every tile of a real block; ghost tiles that hold a live cell
    t.work.clear();
    t.work_slot_begin.assign(nslot + 1, 0);
    t.halo_cells = 0;
    for (int s = 0; s < nslot; ++s) {
      t.work_slot_begin[s] = int32_t(t.work.size());
      for (int tl = 0; tl < t.tiles_per_block; ++tl) {
        bool any = s < t.nreal;
        for (int c = tl * tile; c < (tl + 1) * tile && s >= t.nreal; ++c) {
          const int i = c % n, j = (c / n) % n, k = c / (n * n);
          const int z = axis_zone(i, n) + 3 * axis_zone(j, n) + 9 * axis_zone(k, n);
          if ((t.zmask[s] >> z) & 1u) {
            any = true;
            ++t.halo_cells;
          }
        }
        if (any) t.work.push_back(s * t.tiles_per_block + tl);
      }
    }
    t.work_slot_begin[nslot] = int32_t(t.work.size());
  }

  // coalesced (cell, direction) pairs, for reporting only
  static const int E[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                               {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1},
                               {1, 0, -1}, {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  for (int L = 0; L + 1 < nlev; ++L) {
    LevelTables& t = out[L];
    int64_t pairs = 0;
    for (int s = 0; s < t.nreal; ++s) {
      if (!(t.flags[s] & kHasFine)) continue;
      for (int c = 0; c < n3; ++c) {
        const int ijk[3] = {c % n, (c / n) % n, c / (n * n)};
        for (int a = 1; a < 19; ++a) {
          int o[3];
          for (int ax = 0; ax < 3; ++ax) {
            const int sc = ijk[ax] - E[a][ax];
            o[ax] = sc < 0 ? -1 : (sc >= n ? 1 : 0);
          }
          bool coal = false;
          // the full source and, for edge directions, its two axis projections
          for (int mask = 1; mask < 8 && !coal; ++mask) {
            int d[3];
            bool valid = true;
            for (int ax = 0; ax < 3; ++ax) {
              d[ax] = (mask >> ax) & 1 ? o[ax] : 0;
              if (((mask >> ax) & 1) && E[a][ax] == 0) valid = false;
            }
            if (!valid) continue;
            const int di = (d[0] + 1) + 3 * (d[1] + 1) + 9 * (d[2] + 1);
            if (di != kNbrSelf && t.nbr[size_t(s) * 27 + di] == kNbrFine) coal = true;
          }
          pairs += coal;
        }
      }
    }
    t.coalesced_pairs = pairs;
  }
  return LBM_OK;
}

}  // namespace lbm

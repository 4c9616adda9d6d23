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

bool Forest::outside(int level, int x, int y, int z) const {
  const int p[3] = {x, y, z};
  for (int a = 0; a < 3; ++a)
    if (!periodic[a] && (p[a] < 0 || p[a] >= dims(level, a))) return true;
  return false;
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
            if (outside(L, l.x + dx, l.y + dy, l.z + dz)) continue;
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
          if (outside(l.level, l.x + dx, l.y + dy, l.z + dz)) continue;
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

int Forest::build_from_leaves(const int R_[3], int n_, const bool periodic_[3], const int32_t* leaves, int64_t count,
                              bool balance, std::string& err) {
  for (int a = 0; a < 3; ++a) R[a] = R_[a], periodic[a] = periodic_[a];
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

int Forest::build_from_callback(const int R_[3], int n_, const bool periodic_[3], int max_level_,
                                int (*refine)(int, int, int, int, void*), void* user, std::string& err) {
  for (int a = 0; a < 3; ++a) R[a] = R_[a], periodic[a] = periodic_[a];
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

int Forest::regrid(const int8_t* flags, int64_t count, int max_level_, Forest& out, std::string& err) const {
  int64_t total = 0;
  for (int L = 0; L < num_levels(); ++L) total += int64_t(by_level_[L].size());
  if (count != total) {
    err = "one flag per leaf expected";
    return LBM_E_INVALID;
  }
  out = Forest();
  for (int a = 0; a < 3; ++a) out.R[a] = R[a], out.periodic[a] = periodic[a];
  out.n = n;
  out.leaves_ = leaves_;
  std::unordered_set<uint64_t> coarsen;
  int64_t i = 0;
  for (int L = 0; L < num_levels(); ++L)
    for (const Leaf& l : by_level_[L]) {
      const int8_t fl = flags[i++];
      if (fl > 0 && L < max_level_) out.split(l);
      if (fl < 0 && L > 0) coarsen.insert(block_key(L, l.x, l.y, l.z));
    }
  out.enforce_balance();
  int lmax = 0;
  for (uint64_t k : out.leaves_) lmax = std::max(lmax, unpack(k).level);
  for (int L = lmax; L >= 1; --L) {
    // parents whose 8 children are all leaves flagged for coarsening
    std::vector<Leaf> parents;
    std::unordered_set<uint64_t> seen;
    for (uint64_t k : coarsen) {
      const Leaf c = unpack(k);
      if (c.level != L) continue;
      const Leaf p{L - 1, c.x >> 1, c.y >> 1, c.z >> 1};
      if (!seen.insert(block_key(p.level, p.x, p.y, p.z)).second) continue;
      bool all = true;
      for (int o = 0; o < 8 && all; ++o) {
        const uint64_t ck = block_key(L, 2 * p.x + (o & 1), 2 * p.y + ((o >> 1) & 1), 2 * p.z + (o >> 2));
        all = coarsen.count(ck) && out.leaves_.count(ck);
      }
      if (all) parents.push_back(p);
    }
    for (const Leaf& p : parents) {
      bool ok = true;
      for (int d = 0; d < 27 && ok; ++d) {
        if (d == 13) continue;
        // a leaf finer than L touching the parent's region forbids the merge
        const int qx = p.x + d % 3 - 1, qy = p.y + (d / 3) % 3 - 1, qz = p.z + d / 9 - 1;
        if (out.outside(L - 1, qx, qy, qz)) continue;
        const int cl = out.covering_level(L - 1, qx, qy, qz);
        if (cl > L - 1) {
          // the neighbour position is split: look at its children next to p
          const int wx = wrap(qx, out.dims(L - 1, 0)), wy = wrap(qy, out.dims(L - 1, 1)), wz = wrap(qz, out.dims(L - 1, 2));
          for (int o = 0; o < 8 && ok; ++o) {
            const int cx = 2 * wx + (o & 1), cy = 2 * wy + ((o >> 1) & 1), cz = 2 * wz + (o >> 2);
            // child touches p's region only if it lies on the side facing p
            const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
            if ((dx == 1 && (o & 1)) || (dx == -1 && !(o & 1)) || (dy == 1 && ((o >> 1) & 1)) ||
                (dy == -1 && !((o >> 1) & 1)) || (dz == 1 && (o >> 2)) || (dz == -1 && !(o >> 2)))
              continue;
            if (out.covering_level(L, cx, cy, cz) > L) ok = false;
          }
        }
      }
      if (!ok) continue;
      for (int o = 0; o < 8; ++o)
        out.leaves_.erase(block_key(L, 2 * p.x + (o & 1), 2 * p.y + ((o >> 1) & 1), 2 * p.z + (o >> 2)));
      out.leaves_.insert(block_key(L - 1, p.x, p.y, p.z));
    }
  }
  if (!out.check_cover(err)) return LBM_E_COVER;
  if (!out.balanced()) {
    err = "regrid produced an unbalanced forest";
    return LBM_E_UNBALANCED;
  }
  out.finalize();
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// level tables
// ---------------------------------------------------------------------------

namespace {

struct SlotMap {
  std::unordered_map<uint64_t, int32_t> slot;
  int32_t find(int L, int x, int y, int z) const {
    auto it = slot.find(block_key(L, x, y, z));
    return it == slot.end() ? -1 : it->second;
  }
};

const int kE[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                       {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1},
                       {1, 0, -1}, {-1, 0, 1},  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

}  // namespace

int build_level_tables(const Forest& f, int tile_cells, std::vector<LevelTables>& out, std::string& err) {
  const int n = f.n;
  const int n3 = n * n * n;
  if (tile_cells <= 0 || n3 % tile_cells) {
    err = "tile size does not divide the block";
    return LBM_E_INVALID;
  }
  const int nlev = f.num_levels();
  out.assign(nlev, LevelTables{});
  std::vector<SlotMap> maps(nlev);
  for (int L = 0; L < nlev; ++L) {
    const auto& leaves = f.level_leaves(L);
    for (int b = 0; b < int(leaves.size()); ++b)
      maps[L].slot[block_key(L, leaves[b].x, leaves[b].y, leaves[b].z)] = b;
  }

  for (int L = 0; L < nlev; ++L) {
    LevelTables& t = out[L];
    const auto& leaves = f.level_leaves(L);
    t.level = L;
    t.n = n;
    t.tile = tile_cells;
    t.tiles_per_block = n3 / tile_cells;
    t.nblocks = int(leaves.size());
    t.nbr.assign(size_t(t.nblocks) * 27, 0);
    t.flags.assign(t.nblocks, 0);
    t.fine_index.assign(t.nblocks, -1);
    for (int s = 0; s < t.nblocks; ++s) {
      const Leaf& l = leaves[s];
      uint32_t fl = kAllSameLevel;
      for (int d = 0; d < 27; ++d) {
        if (f.outside(L, l.x + d % 3 - 1, l.y + (d / 3) % 3 - 1, l.z + d / 9 - 1)) {
          t.nbr[size_t(s) * 27 + d] = kNbrWall;
          fl &= ~uint32_t(kAllSameLevel);
          continue;
        }
        const int px = wrap(l.x + d % 3 - 1, f.dims(L, 0)), py = wrap(l.y + (d / 3) % 3 - 1, f.dims(L, 1)),
                  pz = wrap(l.z + d / 9 - 1, f.dims(L, 2));
        const int cl = f.covering_level(L, px, py, pz);
        int32_t v;
        if (cl == L) {
          v = maps[L].find(L, px, py, pz);
        } else if (cl == L + 1) {
          v = kNbrFine;
          fl = (fl & ~uint32_t(kAllSameLevel)) | kHasFine;
        } else if (cl == L - 1) {
          const int32_t ps = maps[L - 1].find(L - 1, px >> 1, py >> 1, pz >> 1);
          if (ps < 0) {
            err = "coarse neighbour without a leaf";
            return LBM_E_UNBALANCED;
          }
          v = kNbrCoarse0 - (ps * 8 + ((px & 1) | ((py & 1) << 1) | ((pz & 1) << 2)));
          fl = (fl & ~uint32_t(kAllSameLevel)) | kHasCoarse;
        } else {
          err = "2:1 balance violated";
          return LBM_E_UNBALANCED;
        }
        t.nbr[size_t(s) * 27 + d] = v;
      }
      t.flags[s] = fl;
      t.coarse_blocks += (fl & kHasCoarse) ? 1 : 0;
      if (fl & kHasFine) {
        // neighbour tables of the 8 virtual level-(L+1) blocks of this block
        const int row = t.fine_blocks++;
        t.fine_index[s] = row;
        t.fine_slot.push_back(s);
        t.fine_nbr.resize(size_t(row + 1) * 8 * 27, -1);
        for (int o = 0; o < 8; ++o) {
          const int vx = 2 * l.x + (o & 1), vy = 2 * l.y + ((o >> 1) & 1), vz = 2 * l.z + (o >> 2);
          for (int d = 0; d < 27; ++d) {
            if (f.outside(L + 1, vx + d % 3 - 1, vy + (d / 3) % 3 - 1, vz + d / 9 - 1)) {
              t.fine_nbr[(size_t(row) * 8 + o) * 27 + d] = kFineWall;
              continue;
            }
            const int px = wrap(vx + d % 3 - 1, f.dims(L + 1, 0)), py = wrap(vy + (d / 3) % 3 - 1, f.dims(L + 1, 1)),
                      pz = wrap(vz + d / 9 - 1, f.dims(L + 1, 2));
            t.fine_nbr[(size_t(row) * 8 + o) * 27 + d] = maps[L + 1].find(L + 1, px, py, pz);
          }
        }
      }
    }
    t.work.resize(size_t(t.nblocks) * t.tiles_per_block);
    for (size_t w = 0; w < t.work.size(); ++w) t.work[w] = int32_t(w);
  }

  // coalesced (cell, direction) pairs: (X, a) is coalesced if X - e_a, or
  // for an edge direction one of its two axis projections, lies in
  // region(L+1).  Only cells on the block's boundary layer can be (their
  // source leaves the block); the list is ordered by row, direction, cell,
  // so that neighbouring threads of the coalescence read neighbouring cells.
  // Whether (X, a) is coalesced depends only on X's position class (low
  // face, inside or high face along each axis) and a.
  if (int64_t(n3) > 65536) {
    err = "cells per block exceed the 16-bit cell index of the coalescence";
    return LBM_E_INVALID;
  }
  std::vector<int> boundary, bclass;  // cells of the block's outer layer, ascending, and their class
  for (int c = 0; c < n3; ++c) {
    const int ijk[3] = {c % n, (c / n) % n, c / (n * n)};
    int cls = 0;
    for (int ax = 2; ax >= 0; --ax) cls = 3 * cls + (ijk[ax] == 0 ? 0 : (ijk[ax] == n - 1 ? 2 : 1));
    if (cls != 13) {
      boundary.push_back(c);
      bclass.push_back(cls);
    }
  }
  for (int L = 0; L + 1 < nlev; ++L) {
    LevelTables& t = out[L];
    int64_t pairs = 0;
    std::vector<std::vector<int32_t>> by_row;  // each row's chunk records
    for (int s = 0; s < t.nblocks; ++s) {
      if (!(t.flags[s] & kHasFine)) continue;
      const int row = t.fine_index[s];
      uint32_t dirs[27];  // per class: bit a set if (X, a) is coalesced
      for (int cls = 0; cls < 27; ++cls) {
        const int pc[3] = {cls % 3, (cls / 3) % 3, cls / 9};
        dirs[cls] = 0;
        for (int a = 1; a < 19; ++a) {
          int o[3];
          for (int ax = 0; ax < 3; ++ax) {
            const int e = kE[a][ax];
            o[ax] = (pc[ax] == 0 && e > 0) ? -1 : ((pc[ax] == 2 && e < 0) ? 1 : 0);
          }
          bool coal = false;
          for (int mask = 1; mask < 8 && !coal; ++mask) {
            int d[3];
            bool valid = true;
            for (int ax = 0; ax < 3; ++ax) {
              d[ax] = (mask >> ax) & 1 ? o[ax] : 0;
              if (((mask >> ax) & 1) && kE[a][ax] == 0) valid = false;
            }
            if (!valid) continue;
            const int di = (d[0] + 1) + 3 * (d[1] + 1) + 9 * (d[2] + 1);
            if (di != kNbrSelf && t.nbr[size_t(s) * 27 + di] == kNbrFine) coal = true;
          }
          if (coal) dirs[cls] |= 1u << a;
        }
      }
      std::vector<int32_t> recs;
      for (int a = 1; a < 19; ++a) {
        const int64_t first = int64_t(t.coal_cells.size());
        for (size_t q = 0; q < boundary.size(); ++q)
          if ((dirs[bclass[q]] >> a) & 1u) t.coal_cells.push_back(uint16_t(boundary[q]));
        const int64_t end = int64_t(t.coal_cells.size());
        pairs += end - first;
        for (int64_t b = first; b < end; b += kCoalChunk) {
          const int64_t cnt = std::min<int64_t>(end - b, kCoalChunk);
          recs.insert(recs.end(), {int32_t(row), int32_t(s), int32_t(b), int32_t(cnt | (int64_t(a) << 16))});
        }
      }
      by_row.push_back(std::move(recs));
    }
    // every row's chunks on one XCD: rows go to the XCD with the fewest
    // chunks so far, then the per-XCD lists are interleaved (position
    // p runs on XCD p % kXcds), the shorter ones padded with empty chunks
    std::vector<std::vector<int32_t>> per_xcd(kXcds);
    for (const auto& recs : by_row) {
      int best = 0;
      for (int x = 1; x < kXcds; ++x)
        if (per_xcd[x].size() < per_xcd[best].size()) best = x;
      per_xcd[best].insert(per_xcd[best].end(), recs.begin(), recs.end());
    }
    size_t longest = 0;
    for (const auto& v : per_xcd) longest = std::max(longest, v.size() / 4);
    for (size_t k = 0; k < longest; ++k)
      for (int x = 0; x < kXcds; ++x) {
        if (4 * k < per_xcd[x].size())
          t.coal_chunks.insert(t.coal_chunks.end(), per_xcd[x].begin() + 4 * k, per_xcd[x].begin() + 4 * k + 4);
        else
          t.coal_chunks.insert(t.coal_chunks.end(), {0, 0, 0, 0});
      }
    t.coalesced_pairs = pairs;
  }
  return LBM_OK;
}

}  // namespace lbm

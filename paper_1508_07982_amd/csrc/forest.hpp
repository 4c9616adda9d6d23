// Host-side forest of octrees and the per-level device tables derived from it.
//
// Section 3.2 / 3.3: uniform periodic root grid, 8-way splits chosen by a
// callback or given as an explicit leaf list, 2:1 balance over face, edge
// and corner neighbours.  Section 4: every block holds n^3 cells.
//
// Device-side view of one level L ("slots"):
//   * real slots [0, nreal): the level-L leaves, canonical (Morton) order;
//   * ghost slots [nreal, nslot): virtual level-L blocks inside level-(L-1)
//     leaves that touch a level-L leaf (face, edge or corner).  Only their
//     cells within Chebyshev distance 2 of a level-L leaf (the two innermost
//     ghost layers, which are streamed but never collided, section 4) are
//     computed; the rest of a ghost block is never written.
// Each slot stores 19 x n^3 PDFs, slot-major: [slot][direction][cell].
#pragma once

#include <cstdint>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace lbm {

constexpr int kNbrSelf = 13;        // index of offset (0,0,0) in the 27-entry table
constexpr int32_t kNbrNone = -1;    // no stored block there (never read by live cells)
constexpr int32_t kNbrFine = -2;    // region of level L+1: values come by coalescence

struct Leaf {
  int level, x, y, z;
};

// Packed key of a block position (level 5 bits, coordinates 19 bits each).
inline uint64_t block_key(int level, int x, int y, int z) {
  return (uint64_t(level) << 57) | (uint64_t(uint32_t(x)) << 38) | (uint64_t(uint32_t(y)) << 19) |
         uint64_t(uint32_t(z));
}

uint64_t morton3(uint32_t x, uint32_t y, uint32_t z);

class Forest {
 public:
  int R[3] = {1, 1, 1};
  int n = 16;
  int max_level = 0;  // deepest level present

  // Build from an explicit leaf list (validated) or from a refine callback.
  // Returns 0 or an LBM_E_* code with `err` set.
  int build_from_leaves(const int R_[3], int n_, const int32_t* leaves, int64_t count, bool balance,
                        std::string& err);
  int build_from_callback(const int R_[3], int n_, int max_level_, int (*refine)(int, int, int, int, void*),
                          void* user, std::string& err);

  // Level of the leaf covering block position p of `level` (wrapped), if
  // that leaf is on `level` or coarser; level + 1 if p is split further.
  int covering_level(int level, int x, int y, int z) const;
  bool is_leaf(int level, int x, int y, int z) const;
  int dims(int level, int axis) const { return R[axis] << level; }

  // Leaves of one level in canonical order.
  const std::vector<Leaf>& level_leaves(int level) const { return by_level_[level]; }
  int num_levels() const { return max_level + 1; }

 private:
  std::unordered_set<uint64_t> leaves_;
  std::vector<std::vector<Leaf>> by_level_;
  void split(const Leaf& l);
  bool check_cover(std::string& err) const;
  bool balanced() const;
  void enforce_balance();
  void finalize();
};

// Tables of one level, ready to copy to the device.
struct LevelTables {
  int level = 0;
  int n = 0;
  int nreal = 0, nghost = 0;
  int tiles_per_block = 0;     // n^3 / tile
  int tile = 0;                // cells per work tile (= threads per workgroup)
  std::vector<int32_t> nbr;           // [slot][27]
  std::vector<uint32_t> zmask;        // [slot] live zones (27 bits)
  std::vector<int32_t> parent;        // [slot] pslot * 8 + octant (ghost), -1 (real)
  std::vector<int32_t> child_ghost;   // [real][8] ghost slot of level L+1 or -1
  std::vector<uint32_t> flags;        // [slot]
  std::vector<int32_t> work;          // slot * tiles_per_block + tile
  std::vector<int32_t> work_slot_begin;  // [slot + 1] prefix into work (per-block launches)
  std::vector<int32_t> ghost_pos;     // [ghost][3]
  int64_t halo_cells = 0;
  int64_t coalesced_pairs = 0;
};

enum SlotFlags : uint32_t {
  kReal = 1u,           // collided interior block
  kAllSameLevel = 2u,   // every neighbour is a real block of this level
  kHasFine = 4u,        // some neighbour lies in region(L+1)
  kHasGhost = 8u,       // some neighbour is a ghost block
};

// Zone of local coordinate c along one axis: 0 = low two layers, 2 = high two
// layers, 1 = in between; the zone index of a cell is zx + 3 zy + 9 zz.
inline int axis_zone(int c, int n) { return c < 2 ? 0 : (c >= n - 2 ? 2 : 1); }

int build_level_tables(const Forest& f, std::vector<LevelTables>& out, std::string& err);

}  // namespace lbm

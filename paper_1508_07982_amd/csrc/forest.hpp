// Host-side forest of octrees and the per-level device tables derived from it.
//
// Section 3.2 / 3.3: uniform root grid, 8-way splits chosen by a callback
// or given as an explicit leaf list, 2:1 balance over face, edge and corner
// neighbours.  Section 4: every block holds n^3 cells.  Each axis is
// periodic or ends in no-slip walls (section 2.2); positions beyond a wall
// are no neighbours.
//
// Device-side view of one level L: slots [0, nblocks) are the level-L leaves
// in canonical (Morton) order; a level buffer is block-major,
// [slot][direction][cell].  Nothing is stored for the fine ghost layers: the
// two streamed halo layers of section 4 are reconstructed on the fly from
// the level's state at the start of the parent step and from the parent
// level (coarse_source in sweep.hpp, coalesce_kernel in kernels.hip).
#pragma once

#include <cstdint>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace lbm {

constexpr int kNbrSelf = 13;        // index of offset (0,0,0) in the 27-entry table
constexpr int32_t kNbrWall = -1;    // beyond a non-periodic end of the domain: no-slip wall
constexpr int32_t kNbrFine = -2;    // region of level L+1: values come by coalescence
constexpr int32_t kNbrCoarse0 = -3; // region of level L-1: entry = kNbrCoarse0 - (pslot * 8 + octant),
                                    // pslot = parent leaf's slot on level L-1, octant = the
                                    // position of this virtual level-L block inside it

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
  bool periodic[3] = {true, true, true};

  // Build from an explicit leaf list (validated) or from a refine callback.
  // Returns 0 or an LBM_E_* code with `err` set.
  int build_from_leaves(const int R_[3], int n_, const bool periodic_[3], const int32_t* leaves, int64_t count,
                        bool balance, std::string& err);
  int build_from_callback(const int R_[3], int n_, const bool periodic_[3], int max_level_,
                          int (*refine)(int, int, int, int, void*), void* user, std::string& err);

  // Whether block position p of `level` lies beyond a non-periodic end.
  bool outside(int level, int x, int y, int z) const;
  // Level of the leaf covering block position p of `level` (wrapped along
  // periodic axes; p must not be outside()), if that leaf is on `level` or
  // coarser; level + 1 if p is split further.
  int covering_level(int level, int x, int y, int z) const;
  bool is_leaf(int level, int x, int y, int z) const;
  int dims(int level, int axis) const { return R[axis] << level; }

  // Dynamic regrid.  flags[i] for the i-th leaf in canonical order: > 0 split
  // it (if below max_level), < 0 merge it with its 7 siblings if all 8 are
  // leaves flagged < 0, 0 keep.  Order: splits, 2:1 balance by further
  // splits, then merges from the finest level down, each only if no leaf
  // finer than the siblings touches their parent.  Returns the new forest.
  int regrid(const int8_t* flags, int64_t count, int max_level_, Forest& out, std::string& err) const;

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

constexpr int32_t kFineWall = -2;  // fine_nbr entry beyond a non-periodic end

// Tables of one level, ready to copy to the device.
// Coalesced pairs per chunk of the coalescence launch (one workgroup, one
// pair per thread); every chunk holds pairs of one direction only, so that
// the direction is uniform over the workgroup.
constexpr int kCoalChunk = 256;
// Workgroups are dispatched round-robin over the chip's 8 XCDs (workgroup b
// to XCD b % 8), each with its own L2.  The chunk list is laid out so that
// all chunks of one block land on one XCD: the block's neighbour tables,
// which each chunk stages, are then fetched from HBM once.
constexpr int kXcds = 8;

struct LevelTables {
  int level = 0;
  int n = 0;
  int nblocks = 0;
  int tiles_per_block = 0;     // n^3 / tile
  int tile = 0;                // cells per work tile (one workgroup of the sweep)
  std::vector<int32_t> nbr;           // [slot][27]: slot, kNbrFine or a coarse code
  std::vector<uint32_t> flags;        // [slot]
  std::vector<int32_t> fine_index;    // [slot]: row of fine_nbr, or -1 without a finer neighbour
  std::vector<int32_t> fine_nbr;      // [row][octant][27]: level-(L+1) slot of the block at offset d
                                      // from the virtual level-(L+1) block (2 b + octant), -1 if
                                      // that position is no level-(L+1) block, kFineWall beyond a
                                      // non-periodic end
  std::vector<int32_t> work;          // slot * tiles_per_block + tile
  std::vector<int32_t> fine_slot;     // [row]: the slot whose fine_nbr row it is
  std::vector<uint16_t> coal_cells;   // cells of the coalesced (cell, direction) pairs, grouped
                                      // by fine_nbr row, then by direction
  std::vector<int32_t> coal_chunks;   // [chunk][4]: fine_nbr row, slot, first pair, count |
                                      // (direction << 16): at most kCoalChunk pairs of one row
                                      // and direction; count 0 marks a padding chunk.  All
                                      // chunks of one row sit at positions equal mod kXcds.
  int64_t coarse_blocks = 0;          // blocks touching level L-1
  int64_t fine_blocks = 0;            // blocks touching level L+1
  int64_t coalesced_pairs = 0;
};

enum SlotFlags : uint32_t {
  kAllSameLevel = 1u,   // every neighbour is a level-L block
  kHasFine = 2u,        // some neighbour lies in region(L+1)
  kHasCoarse = 4u,      // some neighbour lies in region(L-1)
};

// tile_cells: cells per work tile of the sweep (a divisor of n^3).
int build_level_tables(const Forest& f, int tile_cells, std::vector<LevelTables>& out, std::string& err);

}  // namespace lbm

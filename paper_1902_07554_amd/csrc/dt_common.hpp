// Shared device/host definitions for the MI355X Delaunay library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dt.h"

namespace dtk {

// Vertex id of the infinite vertex, and the unused fourth slot of a 2D cell.
constexpr uint32_t INF_V = 0xFFFFFFFFu;
constexpr uint32_t NOSLOT = 0xFFFFFFFEu;
// ploc value of an inserted (or excluded) point; cfwd value of a live cell.
constexpr uint32_t DONE = 0xFFFFFFFFu;
constexpr uint32_t ALIVE = 0xFFFFFFFFu;
constexpr unsigned long long NOKEY = 0xFFFFFFFFFFFFFFFFull;

// Device-side failure bits (ORed into a flag word, read by the host).
enum : uint32_t {
  FAIL_CELL_POOL = 1u << 0,   // cell pool exhausted
  FAIL_EXACT_CAP = 1u << 1,   // exact-arithmetic expansion capacity exceeded
  FAIL_WALK = 1u << 2,        // point-location walk did not terminate
  FAIL_PIVOT = 1u << 3,       // ridge rotation did not close
  FAIL_CAND_CAP = 1u << 4,    // candidate buffer exhausted
  FAIL_HASH = 1u << 5,        // simplex hash table full
  FAIL_OUT_CAP = 1u << 6,     // output buffer too small
  FAIL_NO_PROGRESS = 1u << 7, // a round inserted no point
  FAIL_INVARIANT = 1u << 8,   // internal consistency check
};

// One triangulation cell, all its fields in one 64-byte record so that a
// cell costs one cache line wherever it is touched.
struct alignas(64) Cell {
  uint4 v;                    // vertices (point indices, INF_V = infinite)
  uint4 n;                    // neighbours: cell << 2 | facet index in the neighbour
  unsigned long long spare;   // unused (the bids live in an array of their own)
  unsigned long long cav;     // cavity claim (round-stamped key)
  unsigned long long shell;   // shell claim (round-stamped key)
  unsigned int fwd;           // ALIVE, or the first cell of the star that replaced it
  unsigned int pos;           // position in the cavity list of its inserting candidate
};
static_assert(sizeof(Cell) == 64, "one cache line per cell");

struct Counters {
  unsigned long long pred[4][4];
  unsigned long long cavcells;    // cells placed in cavities (all candidates)  // [orient2, orient3, in2, in3][calls, fp32 ok, fp64 ok, exact]
  unsigned int flags;
  unsigned int cells;             // cells allocated in the pool
  unsigned int ncand;             // candidates this round
  unsigned int inserted;          // points inserted this round
  unsigned int overflow;          // candidates that gave up (cavity too large)
  unsigned int extused;           // cavity extension chunks taken this round
  unsigned int pending;           // active points not yet inserted (this round)
  unsigned int maxcav;            // largest cavity seen
  unsigned int active;            // points to insert
  unsigned int pad;
  // round control, kept on the device so that rounds run back to back
  // without the host in the loop
  unsigned long long remaining;   // points not yet inserted
  unsigned long long done;        // points inserted
  unsigned long long ins_since;   // inserted since the active list was built
  unsigned int thresh;            // priority threshold of the current level
  unsigned int built_thresh;      // threshold the active list was built for
  unsigned int nact;              // length of the active list
  unsigned int rebuild;           // 1: rebuild the active list this round
  unsigned int stall;             // consecutive rounds without an insertion
  unsigned int skip;              // 1: finished or failed; later rounds do nothing
  unsigned int rounds;            // rounds that did work
  unsigned int pad2;
  unsigned long long cand_total;  // candidates over all rounds
  unsigned int last_ins;          // inserted in the last round (diagnostics)
  unsigned int last_cand;         // candidates in the last round (diagnostics)
  // candidates whose cavity outgrew its list this round: the smallest
  // bid key among them; that point may use the pool-sized list next round
  unsigned long long giant_req;
  unsigned int giant_owner;       // point allowed the pool-sized list (DONE: none)
  unsigned int giant_need;        // 1: a request came before the list existed
  unsigned int giant_rounds;      // rounds with a pool-sized-list owner
  unsigned int pad3;
};

}  // namespace dtk

// Encoding of the executor's predecessor entries (deps[] of a plan).
//
// An entry holds the predecessor's subtask index in its low 28 bits.  Panel
// block subtasks that release their successors early (after the look-ahead
// update of the next block's columns, before the update of the rest of
// their tiles) carry two more fields on their own entries:
//   stage  bits 28-29  when the entry is waited for: 0 before the subtask
//                      starts, 1 before its look-ahead update, 2 before the
//                      update of the rest of its tiles (stages 1 and 2 only
//                      occur on panel block subtasks);
//   early  bit 30      the entry needs the predecessor's early release (its
//                      progress word), not its completion flag.
// The streamed panel blocks of an update subtask (pdep) may carry the early
// bit too.  Entries without these bits are plain completion waits.
#pragma once

#include <cstdint>

namespace tqr {

constexpr int32_t DEP_INDEX = (1 << 28) - 1;
constexpr int DEP_STAGE_SHIFT = 28;
constexpr int32_t DEP_STAGE1 = 1 << DEP_STAGE_SHIFT;
constexpr int32_t DEP_STAGE2 = 2 << DEP_STAGE_SHIFT;
constexpr int32_t DEP_EARLY = 1 << 30;

constexpr int32_t dep_index(int32_t d) { return d & DEP_INDEX; }
constexpr int32_t dep_bits(int32_t d) { return d & ~DEP_INDEX; }
constexpr int dep_stage(int32_t d) { return (d >> DEP_STAGE_SHIFT) & 3; }
constexpr bool dep_early(int32_t d) { return (d & DEP_EARLY) != 0; }

// Progress word of a panel block subtask once it has released its
// successors early: 64 epoch + 1 (the update subtasks' progress words count
// their finished blocks in the same form).
constexpr int32_t early_word(int32_t epoch) { return 64 * epoch + 1; }

}  // namespace tqr

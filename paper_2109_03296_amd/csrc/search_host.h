// Host-side pieces of the trajectory search shared by the per-stack launch
// sequence and the batched persistent search: argument checks, the
// per-stack workspace layout and the offset tables.
#pragma once

#include <vector>

#include "kbm_internal.h"

namespace kbm {
namespace srch {

// Workspace per stack: packed planes, tables, flags, top-K state.
struct StackLayout {
    size_t pk_off, pk_bytes, tab_off, tab_bytes, flags_off, stl_off, sti_off, end;
    size_t off_rel, lin_rel, box_rel, mbox_rel, rank_rel;  // in the table block
};

// Addressing mode of a stack's packed planes (see SearchArgs): one 32-bit
// buffer descriptor if they fit, else two halves of the epochs (split =
// T/2) if each fits, else 64-bit addresses.  split = epochs in the first
// group.
struct PlaneMode {
    int am, split;
};
inline PlaneMode plane_mode(int T, int64_t HW) {
    const uint64_t lim = 0xffffffffull, per = 8ull * (uint64_t)HW;
    if (per * (uint64_t)T <= lim) return PlaneMode{1, T};
    if (T >= 2 && per * (uint64_t)(T - T / 2) <= lim) return PlaneMode{2, T / 2};
    return PlaneMode{0, T};
}

// Layout of one stack's block starting at byte `start` of the workspace.
StackLayout layout(const kbm_stack &s, const kbm_search_params &p, size_t start);

// Full validation of a search request (sets the thread's error text).
kbm_status check_search(const kbm_stack *stacks, const kbm_search_params *p,
                        int32_t num_stacks);

// Offset, bounding-box and rank tables of one stack, as laid out in the
// table block of `l` (buf is resized to l.tab_bytes).  Element offsets of
// epochs at or after `split` are relative to epoch `split`.
void make_tables(const kbm_stack &s, const kbm_search_params &p,
                 const StackLayout &l, int split, std::vector<char> &buf);

}  // namespace srch
}  // namespace kbm

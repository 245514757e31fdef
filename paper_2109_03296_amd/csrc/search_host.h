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

// Layout of one stack's block starting at byte `start` of the workspace.
StackLayout layout(const kbm_stack &s, const kbm_search_params &p, size_t start);

// Full validation of a search request (sets the thread's error text).
kbm_status check_search(const kbm_stack *stacks, const kbm_search_params *p,
                        int32_t num_stacks);

// Offset, bounding-box and rank tables of one stack, as laid out in the
// table block of `l` (buf is resized to l.tab_bytes).
void make_tables(const kbm_stack &s, const kbm_search_params &p,
                 const StackLayout &l, std::vector<char> &buf);

}  // namespace srch
}  // namespace kbm

// Search kernels instantiated for exact epoch counts 18..32 and 60 (K <= 8),
// and for 60 epochs of packed planes above 4 GB (two descriptors).
#include "search_kernels.h"

namespace kbm {
namespace srch {

#define KBM_EXACT_CASE(n) \
    case n: launch_chunks<n, 8, true, 1>(a, stream); return true;

bool launch_exact_b(int T, const SearchArgs &a, hipStream_t stream) {
    if (a.K > 8 || a.am == 0) return false;
    if (a.am == 2) {  // packed planes above 4 GB: two descriptors
        if (T != 60) return false;
        launch_chunks<60, 8, true, 2>(a, stream);
        return true;
    }
    switch (T) {
        KBM_EXACT_CASE(18) KBM_EXACT_CASE(19) KBM_EXACT_CASE(20) KBM_EXACT_CASE(21)
        KBM_EXACT_CASE(22) KBM_EXACT_CASE(23) KBM_EXACT_CASE(24) KBM_EXACT_CASE(25)
        KBM_EXACT_CASE(26) KBM_EXACT_CASE(27) KBM_EXACT_CASE(28) KBM_EXACT_CASE(29)
        KBM_EXACT_CASE(30) KBM_EXACT_CASE(31) KBM_EXACT_CASE(32) KBM_EXACT_CASE(60)
        default: return false;
    }
}

}  // namespace srch
}  // namespace kbm

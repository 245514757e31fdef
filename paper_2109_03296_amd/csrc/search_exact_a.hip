// Search kernels instantiated for exact epoch counts 1..17 (K <= 8).
#include "search_kernels.h"

namespace kbm {
namespace srch {

#define KBM_EXACT_CASE(n) \
    case n: launch_chunks<n, 8, true, 1>(a, stream); return true;

bool launch_exact_a(int T, const SearchArgs &a, hipStream_t stream) {
    if (a.K > 8 || a.am != 1) return false;
    switch (T) {
        KBM_EXACT_CASE(1) KBM_EXACT_CASE(2) KBM_EXACT_CASE(3) KBM_EXACT_CASE(4)
        KBM_EXACT_CASE(5) KBM_EXACT_CASE(6) KBM_EXACT_CASE(7) KBM_EXACT_CASE(8)
        KBM_EXACT_CASE(9) KBM_EXACT_CASE(10) KBM_EXACT_CASE(11) KBM_EXACT_CASE(12)
        KBM_EXACT_CASE(13) KBM_EXACT_CASE(14) KBM_EXACT_CASE(15) KBM_EXACT_CASE(16)
        KBM_EXACT_CASE(17)
        default: return false;
    }
}

}  // namespace srch
}  // namespace kbm

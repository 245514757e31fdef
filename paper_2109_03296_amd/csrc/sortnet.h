// Comparator networks that sort N values, built at compile time: halve the
// wires recursively, sort runs of three with a 3-sorter (minimum, median
// and maximum of three, one instruction each), and join halves with
// Batcher's odd-even merge, which is valid for any two run lengths (merge
// the even-indexed and the odd-indexed subsequences, then one layer of
// compare-exchanges between their interleaved results).  Pure constexpr
// C++, so host code can build and check the same networks.
#pragma once

namespace kbm {
namespace net {

constexpr int MAXW = 64;
constexpr int MAXOPS = 768;

struct Op {
    int t, a, b, c;  // t = 0: compare-exchange (min to a, max to b);
                     // t = 1: 3-sorter (min to a, median to b, max to c)
};

struct Net {
    int nops = 0;
    Op op[MAXOPS] = {};
    int out[MAXW] = {};  // out[r]: wire that holds rank r at the end
};

struct Wires {
    int n = 0;
    int w[MAXW] = {};
};

constexpr Wires every_other(const Wires &l, int start) {
    Wires r;
    for (int i = start; i < l.n; i += 2) r.w[r.n++] = l.w[i];
    return r;
}

// Sorted runs A and B (wires in rank order) -> merged run.
constexpr Wires merge(Net &nt, const Wires &A, const Wires &B) {
    if (A.n == 0) return B;
    if (B.n == 0) return A;
    Wires C;
    if (A.n == 1 && B.n == 1) {
        nt.op[nt.nops++] = Op{0, A.w[0], B.w[0], 0};
        C.n = 2;
        C.w[0] = A.w[0];
        C.w[1] = B.w[0];
        return C;
    }
    const Wires E = merge(nt, every_other(A, 0), every_other(B, 0));
    const Wires O = merge(nt, every_other(A, 1), every_other(B, 1));
    C.w[C.n++] = E.w[0];
    for (int i = 0; i < O.n; ++i) {
        if (i + 1 < E.n) {
            nt.op[nt.nops++] = Op{0, O.w[i], E.w[i + 1], 0};
            C.w[C.n++] = O.w[i];
            C.w[C.n++] = E.w[i + 1];
        } else {
            C.w[C.n++] = O.w[i];
        }
    }
    for (int i = O.n + 1; i < E.n; ++i) C.w[C.n++] = E.w[i];
    return C;
}

constexpr Wires sort(Net &nt, const Wires &W) {
    if (W.n <= 1) return W;
    if (W.n == 2) {
        nt.op[nt.nops++] = Op{0, W.w[0], W.w[1], 0};
        return W;
    }
    if (W.n == 3) {
        nt.op[nt.nops++] = Op{1, W.w[0], W.w[1], W.w[2]};
        return W;
    }
    const int m = W.n / 2;
    Wires L, R;
    for (int i = 0; i < W.n; ++i) {
        if (i < m)
            L.w[L.n++] = W.w[i];
        else
            R.w[R.n++] = W.w[i];
    }
    return merge(nt, sort(nt, L), sort(nt, R));
}

constexpr Net make(int n) {
    Net nt;
    Wires W;
    for (int i = 0; i < n; ++i) W.w[W.n++] = i;
    const Wires C = sort(nt, W);
    for (int i = 0; i < n; ++i) nt.out[i] = C.w[i];
    return nt;
}

template <int N>
struct Table {
    static_assert(N >= 1 && N <= MAXW, "network size");
    static constexpr Net net = make(N);
};

}  // namespace net
}  // namespace kbm

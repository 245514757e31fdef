// Host check of the compile-time sorting networks (sortnet.h): every
// network sorts every 0-1 input (0-1 principle: then it sorts every input,
// since compare-exchange and the 3-sorter commute with monotone maps) for
// N up to 20, and sorts random float inputs (with ties) for every N used by
// the kernels.  Prints "N ops status" lines; exit status 1 on a failure.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <utility>

#include "sortnet.h"

using kbm::net::Net;
using kbm::net::Op;

template <class V>
static void run(const Net &nt, V *v) {
    for (int k = 0; k < nt.nops; ++k) {
        const Op o = nt.op[k];
        if (o.t == 0) {
            const V x = std::min(v[o.a], v[o.b]), y = std::max(v[o.a], v[o.b]);
            v[o.a] = x;
            v[o.b] = y;
        } else {
            V s[3] = {v[o.a], v[o.b], v[o.c]};
            std::sort(s, s + 3);
            v[o.a] = s[0];
            v[o.b] = s[1];
            v[o.c] = s[2];
        }
    }
}

template <int N>
static int check() {
    const Net &nt = kbm::net::Table<N>::net;
    int bad = 0;
    // every output wire appears once
    bool seen[N] = {};
    for (int r = 0; r < N; ++r) {
        if (nt.out[r] < 0 || nt.out[r] >= N || seen[nt.out[r]]) bad = 1;
        else seen[nt.out[r]] = true;
    }
    if (N <= 20) {
        for (uint32_t m = 0; m < (1u << N) && !bad; ++m) {
            int v[N];
            for (int i = 0; i < N; ++i) v[i] = (m >> i) & 1;
            run(nt, v);
            for (int r = 1; r < N; ++r)
                if (v[nt.out[r - 1]] > v[nt.out[r]]) bad = 1;
        }
    }
    std::mt19937 g(1234 + N);
    std::uniform_int_distribution<int> d(-8, 8);
    for (int rep = 0; rep < 20000 && !bad; ++rep) {
        float v[N], ref[N];
        for (int i = 0; i < N; ++i) v[i] = ref[i] = (rep & 1) ? d(g) * 0.5f : (float)g() / 7.0f;
        run(nt, v);
        std::sort(ref, ref + N);
        for (int r = 0; r < N; ++r)
            if (v[nt.out[r]] != ref[r]) bad = 1;
    }
    std::printf("%d %d %s\n", N, nt.nops, bad ? "FAIL" : "ok");
    return bad;
}

template <int... Ns>
static int check_all(std::integer_sequence<int, Ns...>) {
    return (check<Ns + 1>() | ...);
}

int main() { return check_all(std::make_integer_sequence<int, 64>{}); }

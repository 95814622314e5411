// Host driver for the sanitizer build of the pattern planning code
// (ahom_plan.cpp): Smith form, plan, twiddles, canonical point and frequency
// orders for a list of matrices read from stdin ("d m11 m12 ... mdd" per
// line).  Checks Q E R = M, e_j | e_{j+1}, |det Q| = |det R| = 1, that the
// canonical orders are permutations of distinct integer vectors, and prints
// one line per matrix ("ok m e..." or "err code").
#include <cstdint>
#include <cstdio>
#include <set>
#include <string>
#include <vector>

#include "../../paper_1605_05712_amd/csrc/ahom_internal.h"

static int64_t det3(int d, const int64_t A[3][3]) {
    if (d == 2) return A[0][0] * A[1][1] - A[0][1] * A[1][0];
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

int main() {
    int d;
    int bad = 0;
    while (std::scanf("%d", &d) == 1) {
        int64_t M[9];
        for (int i = 0; i < d * d; ++i)
            if (std::scanf("%lld", reinterpret_cast<long long*>(&M[i])) != 1) return 2;
        SmithForm sf{};
        std::string err;
        int rc = ahom_smith_form(d, M, &sf, &err);
        if (rc) { std::printf("err %d\n", rc); continue; }
        // Q E R = M
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                int64_t acc = 0;
                for (int k = 0; k < d; ++k) acc += sf.Q[i][k] * sf.e[k] * sf.R[k][j];
                if (acc != M[i * d + j]) { std::printf("QER mismatch\n"); ++bad; }
            }
        for (int k = 0; k + 1 < d; ++k)
            if (sf.e[k + 1] % sf.e[k] != 0) { std::printf("divisibility\n"); ++bad; }
        const int64_t dq = det3(d, sf.Q), dr = det3(d, sf.R);
        if ((dq != 1 && dq != -1) || (dr != 1 && dr != -1)) { std::printf("not unimodular\n"); ++bad; }
        if (sf.m > 1) {
            Plan plan{};
            rc = ahom_build_plan(sf, 256, &plan, &err);
            if (rc) { std::printf("err %d\n", rc); continue; }
            std::vector<double> tw;
            ahom_build_twiddles(&plan, &tw);
            std::vector<int64_t> pts((size_t)sf.m * d), hs((size_t)sf.m * d);
            ahom_canonical_points(sf, pts.data());
            ahom_canonical_freqs(sf, plan.fm, hs.data());
            std::set<std::vector<int64_t>> sp, sh;
            for (int64_t i = 0; i < sf.m; ++i) {
                sp.insert(std::vector<int64_t>(pts.begin() + i * d, pts.begin() + (i + 1) * d));
                sh.insert(std::vector<int64_t>(hs.begin() + i * d, hs.begin() + (i + 1) * d));
            }
            if ((int64_t)sp.size() != sf.m || (int64_t)sh.size() != sf.m) { std::printf("duplicates\n"); ++bad; }
        }
        std::printf("ok %lld", (long long)sf.m);
        for (int k = 0; k < d; ++k) std::printf(" %lld", (long long)sf.e[k]);
        std::printf("\n");
    }
    return bad ? 1 : 0;
}

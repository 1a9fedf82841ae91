// Host harness for the library's Sturm count (sturm_below, compiled for the
// host).  Reads cases from stdin: M x, then a_0..a_{M-1}, then
// b2_0..b2_{M-2} (squared off-diagonals); prints one count per case.
#include <stdio.h>

#include <vector>

#include "../../paper_2305_18643_amd/csrc/lanczos_device.h"

int main() {
    int M;
    double x;
    while (scanf("%d %lf", &M, &x) == 2) {
        std::vector<double> a(M), b2(M > 1 ? M - 1 : 1, 0.0);
        for (int i = 0; i < M; ++i)
            if (scanf("%lf", &a[i]) != 1) return 2;
        for (int i = 0; i + 1 < M; ++i)
            if (scanf("%lf", &b2[i]) != 1) return 2;
        printf("%d\n", qcm::sturm_below(M, a.data(), b2.data(), x));
    }
    return 0;
}

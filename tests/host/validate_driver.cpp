// Drives the host-only validation unit of the C ABI (built with ASan/UBSan by
// tests/test_abi_host.py).  Exit code 0 and "ALL OK" on success.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <limits>

#include "muffin.h"

static int fails = 0;
#define EXPECT(c)                                                         \
    do {                                                                  \
        if (!(c)) { std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } \
    } while (0)

int main() {
    muffin_params p;
    muffin_default_params(&p);
    muffin_shape s = {64, 64, 8, MUFFIN_F32};
    EXPECT(muffin_validate(&s, &p) == MUFFIN_OK);
    EXPECT(muffin_workspace_bytes(&s, &p) > 9u * 4u * 64u * 64u * 8u);
    EXPECT(muffin_validate(nullptr, &p) == MUFFIN_EINVAL);
    EXPECT(muffin_validate(&s, nullptr) == MUFFIN_EINVAL);
    EXPECT(std::strlen(muffin_last_error()) > 0);
    muffin_shape big = {4096, 4096, 64, MUFFIN_F64};
    EXPECT(muffin_validate(&big, &p) == MUFFIN_OK);
    EXPECT(muffin_workspace_bytes(&big, &p) > (size_t)4096 * 4096 * 64 * 8 * 9);
    for (int n : {0, 3, 7, 12, 8192, -8}) {
        muffin_shape b = {n, 64, 8, MUFFIN_F32};
        EXPECT(muffin_validate(&b, &p) < 0);
    }
    muffin_params q = p;
    q.rho_V = std::numeric_limits<double>::quiet_NaN();
    EXPECT(muffin_validate(&s, &q) == MUFFIN_EINVAL);
    q = p;
    q.mu_nu = -0.0;
    EXPECT(muffin_validate(&s, &q) == MUFFIN_OK);
    q = p;
    q.n_s = 9;
    EXPECT(muffin_validate(&s, &q) == MUFFIN_EUNSUPPORTED);
    if (fails == 0) std::printf("ALL OK\n");
    return fails ? 1 : 0;
}

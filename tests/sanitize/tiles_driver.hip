// Runs the library's host-side tile cutting on ragged row-length patterns
// under AddressSanitizer and UndefinedBehaviorSanitizer (host code only,
// built by tests/test_sanitizers.py; no GPU call is made).  Checks that the
// tiles cover the rows in order, that each holds at most `cap` nonzeros or a
// single row, and that each extends as far as the capacity allows.  Exit
// status: the number of failed patterns.
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_1107_0538_amd/csrc/tiles.hpp"

static bool tiles_ok(const std::vector<int>& rp, int cap)
{
    std::vector<int4> t;
    jpcg::build_tiles(rp, cap, t);
    const int n = (int)rp.size() - 1;
    int r = 0;
    for (const int4& d : t) {
        if (d.x != r || d.y <= d.x || d.y > n) return false;
        if (d.z != rp[d.x] || d.w != rp[d.y]) return false;
        if (d.w - d.z > cap && d.y != d.x + 1) return false;
        if (d.y < n && d.w - d.z <= cap && rp[d.y + 1] - d.z <= cap) return false;  // could have taken one more row
        r = d.y;
    }
    return r == n;
}

int main()
{
    std::mt19937 g(7);
    int fails = 0, cases = 0;
    for (int pattern = 0; pattern < 5; ++pattern)
        for (int cap : {256, 512, 1024}) {
            const int n = pattern == 4 ? 1 : 3000;
            std::vector<int> rp(n + 1, 0);
            for (int i = 0; i < n; ++i) {
                int len = 27;
                if (pattern == 1) len = (int)(g() % 61);                 // ragged, some empty rows
                if (pattern == 2) len = i == n / 2 ? 5000 : 8;           // one hub row longer than a tile
                if (pattern == 3) len = (i % 97 == 0) ? cap : (int)(g() % 4);  // rows of exactly one tile
                if (pattern == 4) len = 3;
                rp[i + 1] = rp[i] + len;
            }
            ++cases;
            if (!tiles_ok(rp, cap)) {
                std::printf("FAIL pattern %d cap %d\n", pattern, cap);
                ++fails;
            }
        }
    std::printf("tiles driver: %d of %d patterns failed\n", fails, cases);
    return fails;
}

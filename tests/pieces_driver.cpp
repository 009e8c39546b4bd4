// Test driver: prints the row-piece cap wv_pieces.h chooses for each launch read from stdin.
// Input per launch: strip fill resident ngroups, then ngroups triples h w planes.
#include "../paper_2405_12631_amd/csrc/wv_pieces.h"

#include <cstdio>

int main() {
    int strip, fill, ng;
    long long resident;
    while (std::scanf("%d %d %lld %d", &strip, &fill, &resident, &ng) == 4) {
        std::vector<std::array<int, 3>> shapes((size_t)ng);
        for (auto& s : shapes)
            if (std::scanf("%d %d %d", &s[0], &s[1], &s[2]) != 3) return 1;
        std::printf("%d\n", wv::fused_seg_cap(shapes, strip, fill, resident));
    }
    return 0;
}

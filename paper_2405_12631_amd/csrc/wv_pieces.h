// Row pieces of the fused row-streaming launches (step stacks, ConvLSTM): how a subband's
// rows are cut into work items, and the cut each launch uses.  Host code.
#pragma once

#include <algorithm>
#include <array>
#include <vector>

namespace wv {

// Rows per work item: whole strips up to cap rows, else even pieces of at most cap rows (each
// piece of a step stack recomputes 3 rows of context above and below; a piece of any height
// gives the same outputs).
inline int stack_seg_rows(int h, int cap = 128) {
    const int pieces = (h + cap - 1) / cap;
    return (h + pieces - 1) / pieces;
}

// The piece cap of a fused launch over several plane groups' subbands ({h, w, planes} each):
// the one among a few candidates that minimises the most row steps a resident workgroup walks.
// Items are dealt round-robin over min(items, resident) workgroups in the kernels' order (strip
// fastest, then piece, then plane, group after group), and a piece of R rows costs R + fill row
// steps (fill: 10 for a step stack, 3 for the ConvLSTM).  The strips of one (plane, piece) cost
// the same, so each such run is added to the workgroups it lands on through a difference array
// (whole turns of the deal to every workgroup), O(runs + workgroups) per candidate.
inline int fused_seg_cap(const std::vector<std::array<int, 3>>& shapes, int strip, int fill, long long resident) {
    static const int caps[] = {16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 1024};
    int best_cap = 128;
    long long best = -1;
    std::vector<long long> diff;
    for (int cap : caps) {
        long long total = 0;
        for (const auto& sh : shapes) {
            const int sr = stack_seg_rows(sh[0], cap);
            total += (long long)((sh[1] + strip - 1) / strip) * ((sh[0] + sr - 1) / sr) * sh[2];
        }
        if (total == 0) return 128;
        const long long g = std::min<long long>(total, std::max<long long>(resident, 1));
        diff.assign((size_t)g + 1, 0);
        long long every = 0;   // added to all workgroups
        long long k = 0;       // index of the next item
        for (const auto& sh : shapes) {
            const int h = sh[0], sr = stack_seg_rows(h, cap), sy = (h + sr - 1) / sr;
            const long long sx = (sh[1] + strip - 1) / strip;
            for (int n = 0; n < sh[2]; ++n)
                for (int y = 0; y < sy; ++y) {
                    const long long cost = std::min(sr, h - y * sr) + fill;
                    every += sx / g * cost;
                    const long long r = sx % g, a = k % g;
                    if (r > 0) {
                        if (a + r <= g) {
                            diff[(size_t)a] += cost;
                            diff[(size_t)(a + r)] -= cost;
                        } else {
                            diff[(size_t)a] += cost;
                            diff[(size_t)g] -= cost;
                            diff[0] += cost;
                            diff[(size_t)(a + r - g)] -= cost;
                        }
                    }
                    k += sx;
                }
        }
        long long run = 0, worst = 0;
        for (long long j = 0; j < g; ++j) {
            run += diff[(size_t)j];
            worst = std::max(worst, run);
        }
        worst += every;
        if (best < 0 || worst < best) {
            best = worst;
            best_cap = cap;
        }
    }
    return best_cap;
}

}  // namespace wv

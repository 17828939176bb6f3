// Host-side ordering of one launch's task list for k_gemm_tasks.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

#include "kernels.h"

namespace ep {

// Reorder the tasks of one launch for the XCD-contiguous block mapping (the
// k_gemm_tasks blocks of XCD x run tasks [x per, (x + 1) per) in order): cut
// the emission order, which keeps operand-sharing tasks together, into eight
// contiguous pieces of equal work, put each piece longest task first, and pad
// the pieces to equal length with empty tasks.
inline void balance_xcd(std::vector<GemmTask>& tasks, int64_t off, int64_t& n) {
    if (n <= 0) return;
    auto work = [](const GemmTask& t) {
        int64_t w = 1;
        for (int q = 0; q < ((t.flags >> 4) & 3); q++) w += t.s[q].nk;
        return w;
    };
    std::vector<GemmTask> src(tasks.begin() + off, tasks.begin() + off + n);
    int64_t total = 0;
    for (const GemmTask& t : src) total += work(t);
    std::vector<int64_t> cut(9, (int64_t)src.size());
    cut[0] = 0;
    int64_t acc = 0;
    int c = 1;
    for (int64_t i = 0; i < (int64_t)src.size() && c < 8; i++) {
        acc += work(src[i]);
        while (c < 8 && acc * 8 >= total * c) cut[c++] = i + 1;
    }
    int64_t per = 0;
    for (int x = 0; x < 8; x++) per = std::max(per, cut[x + 1] - cut[x]);
    std::vector<GemmTask> out((size_t)(8 * per), GemmTask{});
    for (int x = 0; x < 8; x++) {
        std::stable_sort(src.begin() + cut[x], src.begin() + cut[x + 1],
                         [&](const GemmTask& a, const GemmTask& b) { return work(a) > work(b); });
        std::copy(src.begin() + cut[x], src.begin() + cut[x + 1], out.begin() + x * per);
    }
    tasks.resize((size_t)off);
    tasks.insert(tasks.end(), out.begin(), out.end());
    n = 8 * per;
}

}  // namespace ep

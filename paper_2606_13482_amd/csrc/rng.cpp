// Row sample of the random-sampling convergence criterion.
//
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the state advances by the
// golden-ratio increment 0x9E3779B97F4A7C15 and each output is the state
// passed through two xor-shift-multiply rounds (multipliers
// 0xBF58476D1CE4E5B9 and 0x94D049BB133111EB, shifts 30, 27, 31).
// Floyd's algorithm (Bentley & Floyd, CACM 1987) picks S distinct integers in
// [0, N): for j from N-S to N-1, draw t uniform on [0, j] and keep t, or j if
// t was already kept.  A uniform integer on [0, j] is the upper 64 bits of
// the 128-bit product of a generator output and j + 1.
#include <algorithm>
#include <unordered_set>

#include "bie_internal.hpp"

namespace bie {

namespace {
struct SplitMix64 {
    uint64_t s;
    explicit SplitMix64(uint64_t seed) : s(seed) {}
    uint64_t operator()()
    {
        s += 0x9E3779B97F4A7C15ULL;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
};
}  // namespace

std::vector<int64_t> rscc_rows(int64_t N, int64_t S, uint64_t seed)
{
    std::vector<int64_t> out;
    if (S >= N) {
        out.resize(N);
        for (int64_t i = 0; i < N; ++i) out[i] = i;
        return out;
    }
    SplitMix64 g(seed);
    std::unordered_set<int64_t> kept;
    kept.reserve(size_t(2 * S));
    for (int64_t j = N - S; j < N; ++j) {
        unsigned __int128 prod = (unsigned __int128)g() * (unsigned __int128)(uint64_t)(j + 1);
        int64_t t = int64_t(uint64_t(prod >> 64));
        if (kept.count(t)) kept.insert(j);
        else kept.insert(t);
    }
    out.assign(kept.begin(), kept.end());
    std::sort(out.begin(), out.end());
    return out;
}

}  // namespace bie

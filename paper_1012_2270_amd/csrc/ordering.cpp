// Row ordering for x locality: Reverse Cuthill-McKee (Cuthill and McKee,
// 1969, with the reversal of George, 1971) on the symmetrised sparsity
// pattern of a square CSR matrix.  The paper orders rows by descending length
// and by AMD to study padding and texture-cache use (Section 4.4.2, Table 7)
// and names orderings that improve the cache use of x as future work
// (Section 5); RCM is the bandwidth-reducing ordering built here in place of
// AMD, which needs third-party code.  Host only, plain C++17.
#include <algorithm>
#include <numeric>
#include <vector>

#include "internal.h"

namespace rg {

// Breadth-first numbering as follows.  Graph: i ~ j when i != j and a_ij or
// a_ji is stored.  Components are started, in turn, from the unnumbered
// vertex of smallest (degree, index); the neighbours of each numbered vertex
// that are still unnumbered are numbered in order of (degree, index).  The
// reverse of that sequence is the result: perm[new] = old.
void rcm_order(int64_t n, const int64_t *rp, const int32_t *col, int32_t *perm) {
    if (n > INT32_MAX) fail(RGCSR_EOVERFLOW, "ordering needs n < 2^31");
    // symmetrised adjacency, each list sorted and without repeats
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = rp[i]; k < rp[i + 1]; k++)
            if (col[k] != i) {
                cnt[i + 1]++;
                cnt[(int64_t)col[k] + 1]++;
            }
    for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    std::vector<int32_t> adj(cnt[n]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = rp[i]; k < rp[i + 1]; k++)
            if (col[k] != i) {
                adj[fill[i]++] = col[k];
                adj[fill[col[k]]++] = (int32_t)i;
            }
    std::vector<int64_t> beg(n + 1, 0);
    int64_t out = 0;
    for (int64_t i = 0; i < n; i++) {
        auto b = adj.begin() + cnt[i], e = adj.begin() + cnt[i + 1];
        std::sort(b, e);
        const int64_t m = std::unique(b, e) - b;
        beg[i] = out;
        std::copy(b, b + m, adj.begin() + out);  // out <= cnt[i]: compaction moves left
        out += m;
    }
    beg[n] = out;
    std::vector<int64_t> deg(n);
    for (int64_t i = 0; i < n; i++) deg[i] = beg[i + 1] - beg[i];
    auto before = [&](int32_t a, int32_t b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; };

    std::vector<int32_t> starts(n);
    std::iota(starts.begin(), starts.end(), 0);
    std::sort(starts.begin(), starts.end(), before);
    std::vector<char> seen(n, 0);
    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<int32_t> nb;
    for (int32_t s : starts) {
        if (seen[s]) continue;
        seen[s] = 1;
        size_t head = order.size();
        order.push_back(s);
        while (head < order.size()) {
            const int32_t v = order[head++];
            nb.clear();
            for (int64_t k = beg[v]; k < beg[v + 1]; k++)
                if (!seen[adj[k]]) nb.push_back(adj[k]);
            std::sort(nb.begin(), nb.end(), before);
            for (int32_t u : nb) {
                seen[u] = 1;
                order.push_back(u);
            }
        }
    }
    for (int64_t i = 0; i < n; i++) perm[i] = order[n - 1 - i];
}

}  // namespace rg

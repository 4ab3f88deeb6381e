// Node orderings of the host setup: the mesh's node adjacency, reverse
// Cuthill-McKee (the paper reorders with RCM to shrink the matrix bandwidth,
// "Software implementation" section) and, for batches, the 3-D Hilbert
// curve.
#include "mdx_host.h"

namespace mdx {
namespace host {

// ---------------------------------------------------------------------------
// graph of the mesh: node -> neighbouring nodes (sharing an element), no
// self.  Elements are 4-id records of which the first npe ids are used.
// ---------------------------------------------------------------------------
void node_graph(int64_t n, int64_t m, int npe, const int32_t *tets, std::vector<int64_t> &ptr,
                std::vector<int32_t> &adj)
{
    std::vector<int64_t> tptr(n + 1, 0);
    for (int64_t e = 0; e < m; ++e)
        for (int a = 0; a < npe; ++a) tptr[tets[4 * e + a] + 1]++;
    for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
    std::vector<int32_t> tlist(tptr[n]);
    {
        std::vector<int64_t> pos(tptr.begin(), tptr.end() - 1);
        for (int64_t e = 0; e < m; ++e)
            for (int a = 0; a < npe; ++a) tlist[pos[tets[4 * e + a]]++] = (int32_t)e;
    }
    std::vector<int32_t> mark(n, -1);
    ptr.assign(n + 1, 0);
    adj.clear();
    adj.reserve((size_t)(14 * n));
    for (int64_t i = 0; i < n; ++i) {
        size_t row0 = adj.size();
        mark[i] = (int32_t)i;
        for (int64_t q = tptr[i]; q < tptr[i + 1]; ++q) {
            const int32_t *t = tets + 4 * (int64_t)tlist[q];
            for (int a = 0; a < npe; ++a)
                if (mark[t[a]] != (int32_t)i) {
                    mark[t[a]] = (int32_t)i;
                    adj.push_back(t[a]);
                }
        }
        std::sort(adj.begin() + row0, adj.end());
        ptr[i + 1] = (int64_t)adj.size();
    }
}

// Reverse Cuthill-McKee: per connected component, BFS from a pseudo-peripheral
// node (George-Liu search) visiting neighbours by increasing degree (ties by
// index); the concatenated order is reversed.  Returns perm[new] = old.
std::vector<int32_t> rcm(int64_t n, const std::vector<int64_t> &ptr, const std::vector<int32_t> &adj)
{
    auto deg = [&](int32_t v) { return ptr[v + 1] - ptr[v]; };
    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<char> placed(n, 0);
    std::vector<int32_t> level(n, -1), queue;
    queue.reserve(n);
    std::vector<int32_t> touched;

    // BFS levels from root; returns eccentricity and the last level's nodes
    auto bfs_levels = [&](int32_t root, std::vector<int32_t> &last) {
        for (int32_t v : touched) level[v] = -1;
        touched.clear();
        queue.clear();
        queue.push_back(root);
        level[root] = 0;
        touched.push_back(root);
        size_t head = 0;
        int ecc = 0;
        while (head < queue.size()) {
            int32_t v = queue[head++];
            ecc = std::max(ecc, level[v]);
            for (int64_t q = ptr[v]; q < ptr[v + 1]; ++q) {
                int32_t w = adj[q];
                if (level[w] < 0) {
                    level[w] = level[v] + 1;
                    touched.push_back(w);
                    queue.push_back(w);
                }
            }
        }
        last.clear();
        for (int32_t v : queue)
            if (level[v] == ecc) last.push_back(v);
        return ecc;
    };

    std::vector<int32_t> last, nbr;
    for (int64_t s = 0; s < n; ++s) {
        if (placed[s]) continue;
        int32_t root = (int32_t)s;
        int ecc = bfs_levels(root, last);
        for (int guard = 0; guard < 64; ++guard) {
            int32_t cand = last[0];
            for (int32_t v : last)
                if (deg(v) < deg(cand) || (deg(v) == deg(cand) && v < cand)) cand = v;
            std::vector<int32_t> last2;
            int e2 = bfs_levels(cand, last2);
            if (e2 > ecc) {
                root = cand;
                ecc = e2;
                last.swap(last2);
            } else {
                break;
            }
        }
        // Cuthill-McKee BFS from root
        size_t head = order.size();
        order.push_back(root);
        placed[root] = 1;
        while (head < order.size()) {
            int32_t v = order[head++];
            nbr.clear();
            for (int64_t q = ptr[v]; q < ptr[v + 1]; ++q)
                if (!placed[adj[q]]) nbr.push_back(adj[q]);
            std::sort(nbr.begin(), nbr.end(), [&](int32_t a, int32_t b) {
                return deg(a) < deg(b) || (deg(a) == deg(b) && a < b);
            });
            for (int32_t w : nbr) {
                placed[w] = 1;
                order.push_back(w);
            }
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// Position of a point on the 3-D Hilbert curve of order `bits` (Skilling's
// transform of the axes to the transposed Hilbert index, then bit
// interleaving): points close on the curve are close in space, so a run of
// consecutive nodes is a compact patch of the mesh.
uint64_t hilbert_key(uint32_t x0, uint32_t x1, uint32_t x2, int bits)
{
    uint32_t X[3] = {x0, x1, x2};
    const uint32_t M = 1u << (bits - 1);
    // inverse undo of the excess work
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    // Gray encode
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t h = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> b) & 1u);
    return h;
}

// nodes [p0, p1) sorted by the Hilbert key of their coordinates in the
// bounding box of that range (2^10 cells per axis)
void hilbert_order(const std::vector<double> &xyz, int64_t p0, int64_t p1,
                   std::vector<int32_t> &out)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = p0; v < p1; ++v)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], xyz[3 * v + k]);
            hi[k] = std::max(hi[k], xyz[3 * v + k]);
        }
    const int bits = 10;
    const double cells = (double)((1u << bits) - 1);
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = std::max(ext, hi[k] - lo[k]);
    const double sc = ext > 0.0 ? cells / ext : 0.0;
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)(p1 - p0));
    for (int64_t v = p0; v < p1; ++v) {
        uint32_t c[3];
        for (int k = 0; k < 3; ++k)
            c[k] = (uint32_t)std::min(cells, std::max(0.0, (xyz[3 * v + k] - lo[k]) * sc));
        key[v - p0] = {hilbert_key(c[0], c[1], c[2], bits), (int32_t)v};
    }
    std::sort(key.begin(), key.end());
    for (auto &kv : key) out.push_back(kv.second);
}

// 16-bit column offsets from each slice's smallest column, when every
// slice's columns span fewer than 2^16 indices

}  // namespace host
}  // namespace mdx

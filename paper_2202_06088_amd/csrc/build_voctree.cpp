// Host-side octree construction over a list of occupied leaf cells.
//
// The leaves are sorted by Morton code (bits of i, j, k interleaved, i in the
// lowest position); a leaf's slot is its rank in that order, so leaves that
// are close in space are close in the payload arrays. The octree is stored
// two levels per node: a node is a cube of 4^3 child cells (2^3 for the root
// when the depth is odd) described by a 64-bit occupancy mask, with the
// occupied children stored consecutively from a base index. Nodes are the
// distinct Morton prefixes of each node level, stored level by level from
// the root (breadth first) and in Morton order within a level, so the top
// levels form a prefix of the table that a kernel can stage in LDS, and the
// children of one node are consecutive rows (or leaf slots).
#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

namespace neuvv {

static inline uint64_t spread3(uint64_t v) {
    // v has at most 21 bits; move bit b to bit 3b
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

static inline uint64_t morton3(uint32_t i, uint32_t j, uint32_t k) {
    return spread3(i) | (spread3(j) << 1) | (spread3(k) << 2);
}

// Returns 0 or a negative neuvv_status; err receives a message.
int build_voctree_host(int32_t depth, int64_t n, const int32_t* ijk, int32_t* nodes, int64_t capacity,
                       int64_t* n_nodes_out, int64_t* slot_of_input, int32_t* box_out, std::string& err) {
    const int64_t G = int64_t(1) << depth;
    std::vector<uint64_t> code(n);
    int32_t box[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t q = 0; q < n; ++q) {
        const int32_t i = ijk[3 * q], j = ijk[3 * q + 1], k = ijk[3 * q + 2];
        if (i < 0 || j < 0 || k < 0 || i >= G || j >= G || k >= G) {
            err = "leaf " + std::to_string(q) + " has a coordinate outside [0, 2^depth)";
            return -2;
        }
        code[q] = morton3((uint32_t)i, (uint32_t)j, (uint32_t)k);
        const int32_t c[3] = {i, j, k};
        for (int a = 0; a < 3; ++a) {
            if (q == 0 || c[a] < box[a]) box[a] = c[a];
            if (q == 0 || c[a] + 1 > box[3 + a]) box[3 + a] = c[a] + 1;
        }
    }
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), int64_t(0));
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return code[a] < code[b]; });
    for (int64_t s = 1; s < n; ++s)
        if (code[order[s]] == code[order[s - 1]]) {
            err = "leaf cell listed twice (inputs " + std::to_string(order[s - 1]) + " and " +
                  std::to_string(order[s]) + ")";
            return -3;
        }
    std::vector<uint64_t> sorted(n);
    for (int64_t s = 0; s < n; ++s) sorted[s] = code[order[s]];

    // node levels: level w covers cubes of edge 2^e[w] split into cells of edge
    // 2^(e[w] - b[w]); b[0] = 1 for odd depth, else 2; b[w > 0] = 2.
    const int L = (depth + 1) / 2;
    std::vector<int> e(L + 1), b(L);
    e[0] = depth;
    for (int w = 0; w < L; ++w) {
        b[w] = (w == 0 && (depth & 1)) ? 1 : 2;
        e[w + 1] = e[w] - b[w];
    }
    // distinct prefixes per level: level w keys = code >> 3 e[w]
    std::vector<std::vector<uint64_t>> keys(L);
    std::vector<int64_t> offset(L + 1, 0);
    for (int w = 0; w < L; ++w) {
        const int sh = 3 * e[w];
        std::vector<uint64_t>& kl = keys[w];
        if (w == 0) {
            kl.push_back(0);
        } else {
            kl.reserve(n ? n : 1);
            for (int64_t s = 0; s < n; ++s) {
                const uint64_t key = sorted[s] >> sh;
                if (kl.empty() || kl.back() != key) kl.push_back(key);
            }
        }
        offset[w + 1] = offset[w] + (int64_t)kl.size();
    }
    const int64_t n_nodes = offset[L];
    if (n_nodes > INT32_MAX || n > INT32_MAX) {
        err = "tree too large for 32-bit node and leaf indices";
        return -2;
    }
    *n_nodes_out = n_nodes;
    if (box_out)
        for (int a = 0; a < 6; ++a) box_out[a] = box[a];
    if (slot_of_input)
        for (int64_t s = 0; s < n; ++s) slot_of_input[order[s]] = s;
    if (!nodes) return 0;
    if (capacity < n_nodes) {
        err = "node_capacity " + std::to_string(capacity) + " < required " + std::to_string(n_nodes);
        return -4;
    }
    std::fill(nodes, nodes + n_nodes * 4, 0);
    // Sets child bit q of node row r; the first child seen (lowest bit, since
    // children arrive in Morton order) fixes the base index.
    auto add_child = [&](int64_t r, int q, int64_t index) {
        int32_t* nd = nodes + r * 4;
        const bool first = nd[0] == 0 && nd[1] == 0;
        if (q < 32) nd[0] = (int32_t)((uint32_t)nd[0] | (1u << q));
        else nd[1] = (int32_t)((uint32_t)nd[1] | (1u << (q - 32)));
        if (first) nd[2] = (int32_t)index;
    };
    // links from level w to level w + 1 (both sorted: parents found by a merge walk)
    for (int w = 0; w + 1 < L; ++w) {
        const std::vector<uint64_t>& up = keys[w];
        const std::vector<uint64_t>& dn = keys[w + 1];
        const int cb = 3 * b[w];
        size_t pu = 0;
        for (size_t q = 0; q < dn.size(); ++q) {
            const uint64_t parent = dn[q] >> cb;
            while (up[pu] != parent) ++pu;
            add_child(offset[w] + (int64_t)pu, (int)(dn[q] & ((1u << cb) - 1)), offset[w + 1] + (int64_t)q);
        }
    }
    // last level: children are leaf slots
    {
        const int w = L - 1;
        const std::vector<uint64_t>& up = keys[w];
        const int cb = 3 * b[w];
        size_t pu = 0;
        for (int64_t s = 0; s < n; ++s) {
            const uint64_t parent = sorted[s] >> cb;
            while (up[pu] != parent) ++pu;
            add_child(offset[w] + (int64_t)pu, (int)(sorted[s] & ((1u << cb) - 1)), s);
        }
    }
    return 0;
}

}  // namespace neuvv

// Host check of a triangle mesh before upload: closed and consistently oriented.
#pragma once
#include <cstdint>
#include <vector>

namespace ibm {

// Every undirected edge must be used by exactly two triangles, once in each direction.  The
// directed edge a -> b becomes the key 2 (min(a, b) nv + max(a, b)) + (a < b); sorted (LSD
// radix, 16-bit digits, as many passes as the largest key needs) the keys of a valid mesh
// come in pairs (2e, 2e + 1).  Returns nullptr, or why the mesh is refused.
inline const char *mesh_closed_oriented(const int32_t *tris, int64_t nt, int64_t nv) {
    const int64_t n = 3 * nt;
    std::vector<uint64_t> a((size_t)n), b((size_t)n);
    for (int64_t t = 0; t < nt; ++t)
        for (int q = 0; q < 3; ++q) {
            const uint64_t u = (uint32_t)tris[3 * t + q], v = (uint32_t)tris[3 * t + (q + 1) % 3];
            if (u == v) return "degenerate edge";
            const uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
            a[(size_t)(3 * t + q)] = 2 * (lo * (uint64_t)nv + hi) + (u < v ? 1u : 0u);
        }
    const uint64_t maxkey = 2 * ((uint64_t)nv * (uint64_t)nv) + 1;  // nv < 2^31: no overflow
    std::vector<int64_t> cnt(65536);
    for (int sh = 0; sh < 64 && (maxkey >> sh) != 0; sh += 16) {
        for (auto &c : cnt) c = 0;
        for (int64_t i = 0; i < n; ++i) ++cnt[(a[(size_t)i] >> sh) & 0xffff];
        int64_t s = 0;
        for (auto &c : cnt) {
            const int64_t c0 = c;
            c = s;
            s += c0;
        }
        for (int64_t i = 0; i < n; ++i) b[(size_t)cnt[(a[(size_t)i] >> sh) & 0xffff]++] = a[(size_t)i];
        a.swap(b);
    }
    for (int64_t i = 0; i < n; i += 2) {
        if (i + 1 >= n) return "mesh is not closed (edge without its reverse)";
        const uint64_t k0 = a[(size_t)i], k1 = a[(size_t)i + 1];
        if ((k0 & 1) == 0 && k1 == k0 + 1) continue;
        if (k1 == k0) return "mesh is not consistently oriented (directed edge used twice)";
        return "mesh is not closed (edge without its reverse)";
    }
    return nullptr;
}

}  // namespace ibm

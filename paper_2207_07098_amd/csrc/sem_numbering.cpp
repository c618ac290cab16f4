// Node numbering from corner ids (see sem_numbering.h).
#include "sem_numbering.h"

#include <algorithm>
#include <unordered_map>
#include <utility>

namespace sem {

// Numbering (Eq. (10): local copies of a physical node share one value).
//
// Each GLL point of an element is classified by how many of its indices sit
// on the element boundary: 3 -> a vertex (keyed by its corner id), 2 -> an
// edge (keyed by the sorted pair of end-vertex ids and the position measured
// from the smaller id), 1 -> a face (keyed by the sorted four corner ids and
// the position in a frame anchored at the smallest id, first axis towards
// the smaller of its two neighbours), 0 -> an element-interior node.  These
// keys depend only on vertex ids, so every element sharing an entity sees
// the same key for the same point whatever its local orientation.  The
// canonical id is the order of first appearance; the solver order puts the
// element-boundary nodes first and the interior nodes after them,
// element by element.

namespace {

struct PairHash {
    size_t operator()(const std::pair<int64_t, int64_t> &p) const {
        uint64_t h = (uint64_t)p.first * 0x9E3779B97F4A7C15ull;
        h ^= (uint64_t)p.second + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
        return (size_t)h;
    }
};
struct Quad {
    int64_t v[4];
    bool operator==(const Quad &o) const {
        return v[0] == o.v[0] && v[1] == o.v[1] && v[2] == o.v[2] && v[3] == o.v[3];
    }
};
struct QuadHash {
    size_t operator()(const Quad &q) const {
        uint64_t h = 1469598103934665603ull;
        for (int a = 0; a < 4; ++a) {
            h ^= (uint64_t)q.v[a] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
            h *= 1099511628211ull;
        }
        return (size_t)h;
    }
};


}  // namespace

int build_numbering(int N, int64_t E, const int64_t *C, const uint8_t *face_bc,
                    int64_t num_vertices, Numbering &out, std::string &err) {
    const int n1 = N + 1, np = n1 * n1 * n1;
    const int nb = np - (N - 1) * (N - 1) * (N - 1);   // points on the element boundary
    const int64_t n_local = E * np;
    auto fail = [&](int code, const std::string &msg) {
        err = msg;
        return code;
    };
    const int ne = N - 1;                    // interior points per edge
    const int nf = ne * ne;                  // interior points per face

    std::unordered_map<std::pair<int64_t, int64_t>, int64_t, PairHash> edges;
    std::unordered_map<Quad, int64_t, QuadHash> faces;
    edges.reserve((size_t)E * 4);
    faces.reserve((size_t)E * 4);
    std::vector<int32_t> edge_gid, face_gid;
    std::vector<int8_t> face_users;
    std::vector<int32_t> vert_gid((size_t)num_vertices, -1);
    if ((double)n_local >= 2147483647.0) return fail(8, "more than 2^31-1 local points");
    out.gid_canon.assign((size_t)n_local, 0);
    std::vector<uint8_t> is_interior;
    std::vector<uint8_t> dir;
    std::vector<int32_t> mult;
    is_interior.reserve((size_t)n_local / 2);
    dir.reserve((size_t)n_local / 2);
    mult.reserve((size_t)n_local / 2);
    int64_t next = 0;
    auto fresh = [&](bool interior) -> int32_t {
        is_interior.push_back(interior);
        dir.push_back(0);
        mult.push_back(0);
        return (int32_t)next++;
    };

    // register faces first to validate conformity (each face used <= 2 times)
    static const int fcorner[6][4] = {{0, 2, 4, 6}, {1, 3, 5, 7}, {0, 1, 4, 5},
                                      {2, 3, 6, 7}, {0, 1, 2, 3}, {4, 5, 6, 7}};
    for (int64_t e = 0; e < E; ++e) {
        const int64_t *v = C + e * 8;
        for (int a = 0; a < 8; ++a) {
            if (v[a] < 0 || v[a] >= num_vertices)
                return fail(2, "element " + std::to_string(e) +
                                                  ": corner id out of range");
            for (int b = 0; b < a; ++b)
                if (v[a] == v[b])
                    return fail(2, "element " + std::to_string(e) +
                                                      ": repeated corner id");
        }
        for (int f = 0; f < 6; ++f) {
            Quad q{{v[fcorner[f][0]], v[fcorner[f][1]], v[fcorner[f][2]], v[fcorner[f][3]]}};
            std::sort(q.v, q.v + 4);
            auto it = faces.find(q);
            if (it == faces.end()) {
                faces.emplace(q, (int64_t)face_users.size());
                face_users.push_back(1);
            } else if (++face_users[it->second] > 2) {
                return fail(2, "face of element " + std::to_string(e) +
                                                  " shared by more than two elements");
            }
        }
    }
    face_gid.assign(face_users.size() * (size_t)nf, -1);

    for (int64_t e = 0; e < E; ++e) {
        const int64_t *v = C + e * 8;
        const uint8_t *fb = face_bc ? face_bc + e * 6 : nullptr;
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    const int l = i + n1 * (j + n1 * k);
                    const int ext[3] = {i == 0 || i == N, j == 0 || j == N, k == 0 || k == N};
                    const int nx = ext[0] + ext[1] + ext[2];
                    int32_t g;
                    if (nx == 3) {
                        int cidx = (i == N) + 2 * (j == N) + 4 * (k == N);
                        int32_t &slot = vert_gid[(size_t)v[cidx]];
                        if (slot < 0) slot = fresh(false);
                        g = slot;
                    } else if (nx == 2) {
                        int d = !ext[0] ? 0 : (!ext[1] ? 1 : 2);
                        int pos = d == 0 ? i : (d == 1 ? j : k);
                        int c0 = (d == 0 ? 0 : (i == N)) + (d == 1 ? 0 : 2 * (j == N)) +
                                 (d == 2 ? 0 : 4 * (k == N));
                        int c1 = c0 + (1 << d);
                        int64_t a = v[c0], b = v[c1];
                        if (a > b) { std::swap(a, b); pos = N - pos; }
                        auto key = std::make_pair(a, b);
                        auto it = edges.find(key);
                        int64_t eidx;
                        if (it == edges.end()) {
                            eidx = (int64_t)edges.size();
                            edges.emplace(key, eidx);
                            edge_gid.resize((size_t)(eidx + 1) * ne, -1);
                        } else {
                            eidx = it->second;
                        }
                        int32_t &slot = edge_gid[(size_t)eidx * ne + (pos - 1)];
                        if (slot < 0) slot = fresh(false);
                        g = slot;
                    } else if (nx == 1) {
                        int d = ext[0] ? 0 : (ext[1] ? 1 : 2);
                        int side = d == 0 ? (i == N) : (d == 1 ? (j == N) : (k == N));
                        int p = d == 0 ? j : i;            // first in-face axis
                        int q = d == 2 ? j : k;            // second in-face axis
                        auto corner = [&](int pa, int qa) -> int64_t {
                            int cc;
                            if (d == 0) cc = side + 2 * pa + 4 * qa;
                            else if (d == 1) cc = 2 * side + pa + 4 * qa;
                            else cc = 4 * side + pa + 2 * qa;
                            return v[cc];
                        };
                        int64_t vv[2][2] = {{corner(0, 0), corner(0, 1)}, {corner(1, 0), corner(1, 1)}};
                        int o1 = 0, o2 = 0;
                        for (int pa = 0; pa < 2; ++pa)
                            for (int qa = 0; qa < 2; ++qa)
                                if (vv[pa][qa] < vv[o1][o2]) { o1 = pa; o2 = qa; }
                        int a1 = o1 ? N - p : p, a2 = o2 ? N - q : q;
                        int s, t;
                        if (vv[1 - o1][o2] < vv[o1][1 - o2]) { s = a1; t = a2; } else { s = a2; t = a1; }
                        Quad key{{vv[0][0], vv[0][1], vv[1][0], vv[1][1]}};
                        std::sort(key.v, key.v + 4);
                        int64_t fidx = faces.find(key)->second;
                        int32_t &slot = face_gid[(size_t)fidx * nf + (s - 1) * ne + (t - 1)];
                        if (slot < 0) slot = fresh(false);
                        g = slot;
                    } else {
                        g = fresh(true);
                    }
                    out.gid_canon[(size_t)e * np + l] = g;
                    mult[g] += 1;
                    if (fb && ((i == 0 && fb[0]) || (i == N && fb[1]) || (j == 0 && fb[2]) ||
                               (j == N && fb[3]) || (k == 0 && fb[4]) || (k == N && fb[5])))
                        dir[g] = 1;
                }
    }
    out.n_unique = next;
    out.dir_canon = std::move(dir);
    out.mult_canon = std::move(mult);
    out.solver_pos.assign((size_t)next, 0);
    int64_t pos = 0, ndir = 0;
    for (int64_t g = 0; g < next; ++g)
        if (!is_interior[g]) out.solver_pos[g] = (int32_t)pos++;
    out.n_bnd = pos;
    for (int64_t g = 0; g < next; ++g) {
        if (is_interior[g]) out.solver_pos[g] = (int32_t)pos++;
        ndir += out.dir_canon[g];
    }
    out.n_dir = ndir;

    // compact boundary map and the node -> copies CSR
    out.bmap.assign((size_t)E * nb, 0);
    out.bdir.assign((size_t)out.n_bnd, 0);
    std::vector<int32_t> count((size_t)out.n_bnd + 1, 0);
    for (int64_t e = 0; e < E; ++e) {
        int b = 0;
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    bool bnd = k == 0 || k == N || i == 0 || i == N || j == 0 || j == N;
                    if (!bnd) continue;
                    int32_t g = out.gid_canon[(size_t)e * np + i + n1 * (j + n1 * k)];
                    int32_t sp = out.solver_pos[g];
                    uint8_t d = out.dir_canon[g];
                    out.bmap[(size_t)e * nb + b] = d ? (int32_t)(sp | 0x80000000u) : sp;
                    out.bdir[sp] = d;
                    count[sp + 1] += 1;
                    ++b;
                }
    }
    out.csr_off.assign((size_t)out.n_bnd + 1, 0);
    for (int64_t g = 0; g < out.n_bnd; ++g) out.csr_off[g + 1] = out.csr_off[g] + count[g + 1];
    out.csr_idx.assign((size_t)E * nb, 0);
    std::vector<int32_t> fill(out.csr_off.begin(), out.csr_off.end() - 1);
    for (int64_t q = 0; q < E * nb; ++q) {
        int32_t sp = out.bmap[q] & 0x7fffffff;
        out.csr_idx[fill[sp]++] = (int32_t)q;
    }
    return 0;
}

}  // namespace sem

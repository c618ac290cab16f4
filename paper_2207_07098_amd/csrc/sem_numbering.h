// Node numbering of a conforming hexahedral mesh from corner ids (host
// code, plain C++17 without HIP, so that it also builds with a host
// compiler under sanitizers).
//
// Karp et al., arXiv 2207.07098, Sec. II-A, Eq. (10): local copies of a
// physical node carry one value; the numbering identifies them.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sem {

struct Numbering {
    int64_t n_unique = 0;             // unique nodes
    int64_t n_bnd = 0;                // unique nodes on element boundaries
    int64_t n_dir = 0;                // masked (Dirichlet) unique nodes
    std::vector<int32_t> gid_canon;   // [E][n_p] canonical first-appearance id
    std::vector<int32_t> solver_pos;  // [n_unique] canonical -> solver order
    std::vector<uint8_t> dir_canon;   // [n_unique] 1 = Dirichlet (canonical order)
    std::vector<int32_t> mult_canon;  // [n_unique] copies per node (canonical order)
    std::vector<int32_t> bmap;        // [E][n_b] solver index of each element-boundary
                                      // point, sign bit set on Dirichlet nodes
    std::vector<int32_t> csr_off;     // [n_bnd + 1] boundary node -> copies
    std::vector<int32_t> csr_idx;     // [E * n_b] compact positions e * n_b + b
    std::vector<uint8_t> bdir;        // [n_bnd] Dirichlet flag in solver order
};

// Numbering for order N of E elements with corner_ids [E][8] (ids in
// [0, num_vertices)) and optional face tags face_bc [E][6] (1 = Dirichlet).
// Element-boundary points of one element are listed in the order: plane
// k = 0, the ring of boundary columns of planes 1..N-1, plane k = N (l order
// within each).  Returns 0, or a sem_status code (2: inconsistent mesh,
// 8: too many points) with a message in err.
int build_numbering(int N, int64_t E, const int64_t *corner_ids, const uint8_t *face_bc,
                    int64_t num_vertices, Numbering &out, std::string &err);

}  // namespace sem

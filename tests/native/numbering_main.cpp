// Host driver of the library's numbering (sem_numbering.cpp) for sanitizer
// runs: reads a mesh written by the test suite, numbers it, and writes the
// result for the test to compare with the oracle's lattice numbering.
//
// input  (argv[1]): int32 N, int64 E, int64 num_vertices, int64 corner_ids
//                   [E][8], uint8 face_bc [E][6]
// output (argv[2]): int32 status, int64 n_unique, n_bnd, n_dir, then
//                   gid_canon [E*(N+1)^3] int32, solver_pos [n_unique] int32,
//                   dir_canon [n_unique] uint8, mult_canon [n_unique] int32,
//                   bmap [E*n_b] int32, csr_off [n_bnd+1] int32,
//                   csr_idx [E*n_b] int32, bdir [n_bnd] uint8
// On a numbering error the output holds only the status and the message
// is printed.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "sem_numbering.h"

template <typename T>
static bool rd(FILE *f, T *p, size_t n) { return std::fread(p, sizeof(T), n, f) == n; }
template <typename T>
static void wr(FILE *f, const T *p, size_t n) {
    if (n && std::fwrite(p, sizeof(T), n, f) != n) std::exit(3);
}

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t N = 0;
    int64_t E = 0, nv = 0;
    if (!rd(f, &N, 1) || !rd(f, &E, 1) || !rd(f, &nv, 1) || E < 1 || N < 1) return 2;
    std::vector<int64_t> corners((size_t)E * 8);
    std::vector<uint8_t> fbc((size_t)E * 6);
    if (!rd(f, corners.data(), corners.size()) || !rd(f, fbc.data(), fbc.size())) return 2;
    std::fclose(f);
    sem::Numbering num;
    std::string err;
    const int32_t st = sem::build_numbering(N, E, corners.data(), fbc.data(), nv, num, err);
    FILE *o = std::fopen(argv[2], "wb");
    if (!o) return 2;
    wr(o, &st, 1);
    if (st != 0) {
        std::printf("numbering error %d: %s\n", st, err.c_str());
        std::fclose(o);
        return 0;
    }
    wr(o, &num.n_unique, 1);
    wr(o, &num.n_bnd, 1);
    wr(o, &num.n_dir, 1);
    wr(o, num.gid_canon.data(), num.gid_canon.size());
    wr(o, num.solver_pos.data(), num.solver_pos.size());
    wr(o, num.dir_canon.data(), num.dir_canon.size());
    wr(o, num.mult_canon.data(), num.mult_canon.size());
    wr(o, num.bmap.data(), num.bmap.size());
    wr(o, num.csr_off.data(), num.csr_off.size());
    wr(o, num.csr_idx.data(), num.csr_idx.size());
    wr(o, num.bdir.data(), num.bdir.size());
    std::fclose(o);
    std::printf("numbering ok: n_unique %lld\n", (long long)num.n_unique);
    return 0;
}

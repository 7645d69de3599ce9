// Host-side construction of the screening tables (built once per Hamiltonian).
//
//  * Heat-bath doubles table: for every spin-orbital pair i<j, the tuples
//    (a<b, v = <ab|ij> - <ab|ji>) with |v| > eps, sorted by descending |v|
//    (ties by a, then b), following the section "Reduced scaling evaluation
//    of the local energy".  Candidates are generated from the symmetric images
//    of the non-zero integrals, so the build costs O(n_nz log n_nz) rather than
//    a loop over all quadruples.
//  * Singles: for every spin-orbital i, the same-spin a with
//    S_ia = |h_ia| + sum_j |(ia|jj) - (ij|ja)| > eps (same section), sorted by
//    descending S_ia (ties by a); per entry the vector V_ia[j] = (ia|jj) -
//    delta_{spin i, spin j} (ij|ja) over all spin-orbitals j, so that
//    H_NM = h_ia + sum_{j occupied} V_ia[j].
//  * Diagonal: D_ij = (ii|jj) - delta_{spin} (ij|ji) and h_ii, so that
//    H_NN = sum_i h_ii + sum_{i<j} D_ij.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace vmc {

struct HostTables {
    int n = 0, n_so = 0, na = 0, nb = 0, ne = 0;
    double eps = 0.0;
    std::vector<int64_t> row_off;  // n_so*n_so + 1, row of pair (i<j) at index i*n_so + j
    std::vector<int32_t> dab;      // 2 per entry: a, b
    std::vector<double> dv;        // per entry
    std::vector<int64_t> s_off;    // n_so + 1
    std::vector<int32_t> sa;       // per singles entry
    std::vector<double> sS;        // S_ia per singles entry
    std::vector<double> sh;        // h_ia per singles entry
    std::vector<double> sV;        // n_so per singles entry, j-major within each orbital's row
    std::vector<double> D;         // n_so * n_so
    std::vector<double> hdiag;     // n_so
};

// Returns an empty string on success, else an error message.
std::string build_host_tables(int n, int na, int nb, const double* h1, int64_t n_nz, const int32_t* pqrs,
                              const double* val, double eps, HostTables& out);

}  // namespace vmc

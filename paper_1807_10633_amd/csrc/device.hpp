// Device-side helpers shared by the gfx950 kernels: wave-64 reductions and
// scans, the Philox4x64-10 counter-based generator, and the views of the
// tables and walker buffers that kernels receive by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vmc {

constexpr int kWave = 64;
constexpr int kQueue = 128;  // per-wave survivor queue (<= 63 left over + 64 new)

// ------------------------------------------------------------------ views
struct Tab {
    int n_so, ne, nw, G;
    int n, na;                // spatial orbitals, alpha electrons
    int uhf;                  // spin-blocked orbitals: slots [0, na) alpha, [na, ne) beta
    int rrow;                 // length of one slot's row of R: n_so, or n when uhf (own spin only)
    int has_doubles;          // the table holds at least one doubles entry
    int has_sV;               // some singles entry has a nonzero Coulomb-exchange vector
    int fock;                 // keep the walker's singles elements in its scratch (state in HBM, has_sV)
    double eps;
    double small_den;         // Sherman-Morrison denominators below this in magnitude flag the walker (and
                              // re-invert it after the move where the sweep re-inverts in place)
    uint64_t ham_id;          // identifies this system's Hamiltonian tables (never 0) in the scratch's
                              // singles-element tag
    const uint32_t* row_off;  // n_so*n_so + 1
    const uint32_t* dab;      // a | b << 16
    const uint64_t* dmask;    // (1 << a) | (1 << b) per doubles entry when n_so <= 64, else null
    const double* dvK;        // per doubles entry: <ab||ij>, then exp(Jastrow constant part)
    const uint32_t* s_off;    // n_so + 1
    const uint32_t* sa;       // target orbital a
    const double* sh;         // h_ia
    const double* sV;         // n_so per entry; row of orbital i: V_e[j] at s_off[i] n_so + j len_i + e
    const double* sK;         // exp(J_aa - J_ii - J_ai) per singles entry
    const double* D;          // n_so*n_so
    const double* hdiag;      // n_so
    const double* J;          // dense n_so*n_so
    const double* theta;      // n_so*n_so row-major
    // correlator product state (ncorr = 0: none)
    int ncorr;
    const int32_t* csite;     // 5 per correlator: its sites (spatial orbitals), -1 after the last
    const int32_t* coff;      // ncorr + 1: offsets of each correlator's 4^k coefficients
    const double* cc;         // the coefficients
    const int32_t* sc_off;    // n + 1: the correlators holding each site are sc_list[sc_off[s] ..)
    const uint32_t* sc_list;  // correlator index (low 24 bits) | position of the site in it << 24
};

struct Wk {
    uint64_t* occ;
    int32_t* slot_orb;
    int32_t* orb_slot;
    double* B;
    void* R;  // double (FP64 form) or float (mixed form)
    uint16_t* Rlo;  // mixed form: bfloat16 remainder of each R entry (R = hi + lo), R's layout
    double* s;
    double* hnn;
    double* eloc;
    double* tres;
    int64_t* pick;
    uint32_t* status;
    uint8_t* scratch;
    int64_t scratch_stride;  // bytes per walker
};

// ------------------------------------------------------- wave primitives
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ uint32_t mask_below(uint64_t m) {
    // number of set bits of m strictly below this lane
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Sum over the wave, identical in every lane (lane 0's butterfly result).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    return __shfl(x, 0, kWave);
}

// Inclusive prefix sum over the wave (lane order).
__device__ __forceinline__ double wave_inclusive_scan(double x) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        double y = __shfl_up(x, d, kWave);
        if (l >= d) x += y;
    }
    return x;
}

// --------------------------------------------------------------- Philox
// Philox4x64-10 block function (Salmon, Moraes, Dror and Shaw, SC'11):
// ten rounds of two 64x64->128 multiplies with a Weyl-sequence key schedule.
__device__ __forceinline__ uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                                 uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    return c0;
}

// u in [0,1) for (seed, walker, step): 53 high bits of word 0.
__device__ __forceinline__ double ctmc_uniform(uint64_t seed, uint64_t walker, uint64_t step) {
    const uint64_t x = philox_word0(step, 0, 0, 0, seed, walker);
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ int64_t pack_pick(int type, int i, int j, int a, int b) {
    if (type == 0) return 0;
    const int64_t jj = (type == 2) ? j : 0xFFF, bb = (type == 2) ? b : 0xFFF;
    return ((int64_t)type << 48) | ((int64_t)i << 36) | (jj << 24) | ((int64_t)a << 12) | bb;
}

}  // namespace vmc

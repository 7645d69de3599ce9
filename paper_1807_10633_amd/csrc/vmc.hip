// gfx950 kernels and the C ABI of the screened orbital-space VMC hot path.
//
// One workgroup owns one walker.  Per CTMC step (Sabzevari & Sharma, sections
// "Reduced scaling evaluation of the local energy", "Continuous time Monte
// Carlo" and "Local energy and Gradient ratios"):
//   1. candidate groups (singles of each occupied i; heat-bath row of each
//      occupied pair i<j) are distributed round-robin over the wavefronts;
//      a wave scans a group 64 entries at a time, keeps the entries whose
//      target orbitals are empty (ballot + mbcnt compaction into an LDS
//      queue, order preserving) and evaluates full batches of 64 survivors:
//      ratio = det-ratio (R entry or 2x2 minor of R) x Jastrow ratio, local
//      energy term H_NM x ratio and rate |ratio|;
//   2. per-group rate sums give T = sum r in canonical order; the group
//      holding u*T is found by a chunked prefix sum and re-walked by one wave
//      with a wave-level inclusive scan to locate the picked candidate;
//   3. rank-1 (single) or rank-2 (double) Sherman-Morrison updates of B and R,
//      the Jastrow sums s and the occupation;
//   4. every refresh_period steps B is rebuilt by Gauss-Jordan elimination
//      with partial pivoting and R = theta[:, 0:Ne] B.
// When R, B and the group sums fit in LDS the walker stays on chip for the
// whole multi-step launch; otherwise they live in the caller's buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "device.hpp"
#include "tables.hpp"
#include "vmc.h"


using namespace vmc;

// =============================================================================
// Device code
// =============================================================================
namespace {

struct OccReg {
    uint64_t w;
    __device__ __forceinline__ bool empty(int p) const { return ((w >> p) & 1ull) == 0ull; }
};
struct OccLds {
    const uint64_t* w;
    __device__ __forceinline__ bool empty(int p) const { return ((w[p >> 6] >> (p & 63)) & 1ull) == 0ull; }
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Decode the lexicographic index t of an occupied pair (x<y) among ne slots.
__device__ __forceinline__ void pair_decode(int t, int ne, int& x, int& y) {
    const double b = 2.0 * ne - 1.0;
    int xx = (int)floor((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
    if (xx < 0) xx = 0;
    while (xx > 0 && xx * (2 * ne - xx - 1) / 2 > t) --xx;
    while ((xx + 1) * (2 * ne - xx - 2) / 2 <= t) ++xx;
    x = xx;
    y = t - xx * (2 * ne - xx - 1) / 2 + xx + 1;
}

// Scan entries [base, base+len) of a singles list or heat-bath row, keep
// those whose target orbitals are empty and hand them to eval in batches of
// up to 64 (canonical order).  eval(e, active) returns true to stop early
// (wave-uniform).
template <bool DOUBLES, class Occ, class Eval>
__device__ __forceinline__ void scan_group(const Tab& T, const Occ& occ, uint32_t base, uint32_t len,
                                           uint32_t* queue, Eval& eval) {
    const int l = lane_id();
    uint32_t qn = 0;
    bool stop = false;
    for (uint32_t c = 0; c < len && !stop; c += kWave) {
        const uint32_t e = c + (uint32_t)l;
        bool surv = false;
        if (e < len) {
            if (DOUBLES) {
                const uint32_t ab = T.dab[base + e];
                surv = occ.empty((int)(ab & 0xFFFFu)) && occ.empty((int)(ab >> 16));
            } else {
                surv = occ.empty((int)T.sa[base + e]);
            }
        }
        const uint64_t m = __ballot(surv);
        if (surv) queue[qn + mask_below(m)] = e;
        qn += (uint32_t)__popcll(m);
        if (qn >= (uint32_t)kWave) {
            wave_lds_sync();
            const uint32_t mine = queue[l];
            const uint32_t rest = ((uint32_t)l + kWave < qn) ? queue[l + kWave] : 0u;
            wave_lds_sync();
            qn -= kWave;
            if ((uint32_t)l < qn) queue[l] = rest;
            stop = eval(mine, true);
        }
    }
    if (!stop && qn > 0) {
        wave_lds_sync();
        const uint32_t mine = ((uint32_t)l < qn) ? queue[l] : 0u;
        eval(mine, (uint32_t)l < qn);
    }
    wave_lds_sync();
}

// Group descriptor (wave-uniform).
struct Group {
    int type;  // 1 singles, 2 doubles
    int i, j, p, q;
    uint32_t base, len;
    double fac;  // exp(-s_i) [exp(-s_j)]
};

__device__ __forceinline__ Group group_of(const Tab& T, int g, const int* occl, const int* oslot, const double* ies) {
    Group G;
    const int ne = T.ne, n_so = T.n_so;
    if (g < ne) {
        G.type = 1;
        G.i = occl[g];
        G.j = -1;
        G.p = oslot[G.i];
        G.q = -1;
        G.base = T.s_off[G.i];
        G.len = T.s_off[G.i + 1] - G.base;
        G.fac = ies[G.i];
    } else {
        int x, y;
        pair_decode(g - ne, ne, x, y);
        G.type = 2;
        G.i = occl[x];
        G.j = occl[y];
        G.p = oslot[G.i];
        G.q = oslot[G.j];
        const int row = G.i * n_so + G.j;
        G.base = T.row_off[row];
        G.len = T.row_off[row + 1] - G.base;
        G.fac = ies[G.i] * ies[G.j];
    }
    return G;
}

// Position of R[a][p] in a walker's R: row p (one per slot) holds every
// orbital, or with spin-blocked orbitals only the n orbitals of the slot's own
// spin (slots [0, na) alpha, [na, Ne) beta; a must have that spin).
__device__ __forceinline__ int r_index_uhf(const Tab& T, int p, int a) {
    return p * T.n + a - ((p >= T.na) ? T.n : 0);
}
__device__ __forceinline__ int r_index(const Tab& T, int p, int a) {
    return T.uhf ? r_index_uhf(T, p, a) : p * T.n_so + a;
}
// 2x2 minor from its four gathered FP64 entries of R, with the first product
// fused in one fixed form, so that every evaluation of a candidate rounds
// alike.  (FP32 entries need no such care: their products are exact in FP64,
// and the difference is rounded once however it is contracted.)
__device__ __forceinline__ double minor_of(double rpa, double rqb, double rpb, double rqa) {
    return fma(rpa, rqb, -(rpb * rqa));
}
// 2x2 minor R[a][p] R[b][q] - R[b][p] R[a][q] of a double (section "Local
// energy and Gradient ratios", Eq. eq:R).  Spin-blocked orbitals: a pair of
// the same spin is the full minor within that spin's rows; a pair of opposite
// spins (i alpha, j beta, hence a alpha, b beta) has no cross term, so the
// ratio is the product of the two spins' single ratios.  Products and the
// difference are formed in FP64 whatever the storage of R, so that the
// cancellation of a minor near a node adds no rounding of the storage type.
template <typename RT>
__device__ __forceinline__ double pair_minor_uhf(const Tab& T, const RT* R, int p, int q, int a, int b) {
    const int op = (p >= T.na) ? T.n : 0, oq = (q >= T.na) ? T.n : 0;
    const int rp = p * T.n - op, rq = q * T.n - oq;
    if (op != oq) return (double)R[rp + a] * (double)R[rq + b];
    if constexpr (sizeof(RT) == 8) return minor_of(R[rp + a], R[rq + b], R[rp + b], R[rq + a]);
    return (double)R[rp + a] * (double)R[rq + b] - (double)R[rp + b] * (double)R[rq + a];
}
template <typename RT>
__device__ __forceinline__ double pair_minor(const Tab& T, const RT* R, int p, int q, int a, int b) {
    if (T.uhf) return pair_minor_uhf(T, R, p, q, a, b);
    const RT* Rp = R + p * T.n_so;
    const RT* Rq = R + q * T.n_so;
    return (double)Rp[a] * (double)Rq[b] - (double)Rp[b] * (double)Rq[a];
}

// Ratio and matrix element of candidate e of group Gr (slot convention).
__device__ __forceinline__ double cps_ratio(const Tab& T, const uint32_t* cidx, const double* cinv, int nk, int o0,
                                            int o1, int o2, int o3);
template <typename RT>
__device__ __forceinline__ double single_ratio(const Tab& T, const Group& Gr, uint32_t e, const RT* R,
                                               const double* es, const uint32_t* cidx, const double* cinv, int& a) {
    a = (int)T.sa[Gr.base + e];
    double r = (double)R[r_index(T, Gr.p, a)] * es[a] * Gr.fac * T.sK[Gr.base + e];
    if (T.ncorr) r *= cps_ratio(T, cidx, cinv, 2, Gr.i, a, 0, 0);
    return r;
}
__device__ __forceinline__ double single_h(const Tab& T, const Group& Gr, uint32_t e, const int* occl) {
    const double* V = T.sV + (size_t)Gr.base * T.n_so + e;
    double h = T.sh[Gr.base + e];
    for (int y = 0; y < T.ne; ++y) h += V[(size_t)occl[y] * Gr.len];
    return h;
}
template <typename RT>
__device__ __forceinline__ double double_ratio(const Tab& T, const Group& Gr, uint32_t e, const RT* R,
                                               const double* es, const uint32_t* cidx, const double* cinv, int& a,
                                               int& b) {
    const uint32_t ab = T.dab[Gr.base + e];
    a = (int)(ab & 0xFFFFu);
    b = (int)(ab >> 16);
    const double det = pair_minor(T, R, Gr.p, Gr.q, a, b);
    double r = det * es[a] * es[b] * T.dvK[2 * (size_t)(Gr.base + e) + 1] * Gr.fac;
    if (T.ncorr) r *= cps_ratio(T, cidx, cinv, 4, Gr.i, Gr.j, a, b);
    return r;
}

// --------------------------------------------------------------- LDS layout
constexpr int kLogS = 32;   // batch-log entries per wave, singles stream
constexpr int kLogD = 64;   // batch-log entries per wave, doubles stream
constexpr int kLogGran = 2; // initial batches per log entry
constexpr int kUnroll = 6;  // 64-entry chunks whose table loads are issued together
constexpr int kTileUnroll = 8;  // the same in pair_tiles (measured: 4 is 2 % slower, 8 0.3–0.6 % faster than 6)

struct Lds {
    uint32_t occw, occl, slot, oslot, s, es, ies, red, stmp, mi, md, wst, wtot, q64, qab, lsum, loff, lg, sgend, sdelta,
        svend, spq, sfac, sies, dgend, ddelta, dvend, dpq, dfac, w1, w2, cRp, cRq, cBp, cBq, ipiv, dblk, fcol, cidx, cinv, mark, R,
        B, Rh, thl, total;
};
__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }
// Doubles of the layout with the walker state in HBM run over tiles of
// kPairBlock x kPairBlock occupied pairs (pair_tiles).  32 measured 3 %
// faster than 16 at 160 orbitals (fewer segments, each reduced once), 8
// 4 % slower, 64 the same as 32.
constexpr int kPairBlock = 32;
__host__ __device__ inline int pair_blocks(int ne) { return (ne + kPairBlock - 1) / kPairBlock; }
// rb: bytes per R element (8 for the FP64 form, 4 for the mixed form);
// ncorr: correlators (their current states and inverse coefficients)
__host__ __device__ __forceinline__ Lds lds_layout(int n_so, int ne, int nw, int nt, bool small, int rb, int ncorr) {
    Lds L;
    size_t o = 0;
    const int nwv = nt / 64;
    const size_t gd = (size_t)ne * (ne - 1) / 2;
    auto take = [&](size_t bytes) { const size_t r = o; o += al16(bytes); return (uint32_t)r; };
    L.occw = take((size_t)nw * 8);
    L.occl = take((size_t)ne * 4);
    L.slot = take((size_t)ne * 4);
    L.oslot = take((size_t)n_so * 4);
    L.s = take((size_t)n_so * 8);
    L.es = take((size_t)n_so * 8);
    L.ies = take((size_t)n_so * 8);
    L.red = take((size_t)(nwv + 2) * 8);
    L.stmp = take((size_t)(nt + 1) * 4);
    L.mi = take((size_t)(32 + nwv) * 4);
    L.md = take((size_t)16 * 8);
    L.wst = take((size_t)nwv * 8 * 4);
    L.wtot = take((size_t)nwv * 2 * 8);
    L.q64 = take((size_t)nwv * kQueue * 8);
    L.qab = take((size_t)nwv * kQueue * 8);
    L.lsum = take((size_t)nwv * (kLogS + kLogD) * 8);
    L.loff = take((size_t)nwv * (kLogS + kLogD) * 4);
    L.lg = take((size_t)nwv * (kLogS + kLogD) * 4);
    L.sgend = take((size_t)ne * 4);
    L.sdelta = take((size_t)ne * 4);
    L.svend = take((size_t)ne * 4);
    L.spq = take((size_t)ne * 4);
    L.sfac = take((size_t)ne * 8);
    L.sies = take((size_t)ne * 8);
    L.w1 = take((size_t)ne * 8);
    L.w2 = take((size_t)ne * 8);
    L.cRp = take((size_t)n_so * 8);
    L.cRq = take((size_t)n_so * 8);
    L.cBp = take((size_t)ne * 8);
    L.cBq = take((size_t)ne * 8);
    L.ipiv = take((size_t)ne * 4);
    L.dblk = take(((gd + 63) / 64 + 1) * 4);
    L.fcol = take((size_t)ne * 8);
    L.cidx = take((size_t)ncorr * 4);
    L.cinv = take((size_t)ncorr * 8);
    // state in HBM: per wave, the marker bytes of pair_tiles' row lookup
    L.mark = small ? 0u : take((size_t)nwv * kTileUnroll * 64);
    if (small) {
        L.dgend = take(gd * 4);
        L.ddelta = take(gd * 4);
        L.dvend = take(gd * 4);
        L.dpq = take(gd * 4);
        L.dfac = 0;
        L.R = take((size_t)n_so * ne * rb);
        L.B = take((size_t)ne * ne * 8);
        L.Rh = take((size_t)n_so * ne * rb);
        // mixed form: theta[:, 0:Ne] (FP64) for the per-move GEMM and the FP64 rows
        L.thl = (rb < 8) ? take((size_t)n_so * ne * 8) : 0u;
    } else {
        L.dgend = L.ddelta = L.dvend = L.dpq = L.dfac = L.R = L.B = L.Rh = L.thl = 0;
    }
    L.total = (uint32_t)o;
    return L;
}
// per-walker global scratch (walker state in HBM): the rate sums of the
// doubles' pair segments (Ne x pair_blocks(Ne)), then the tag of the singles
// elements (the nw occupation words they hold, the Hamiltonian's id (0: none)
// and the moves applied to them since they were last built), followed, when
// the singles carry Coulomb-exchange vectors, by the walker's Fock-like
// singles elements (one double per singles-table entry).  The elements depend
// on the occupation and the Hamiltonian only, so a launch whose walker matches
// the tag reuses them; they are rebuilt after kFockRebuild moves so that the
// rounding of the per-move updates stays bounded.
constexpr uint64_t kFockRebuild = 4096;
__host__ __device__ inline size_t scratch_tag_offset(int ne) { return al16((size_t)ne * pair_blocks(ne) * 8 + 16); }
__host__ __device__ inline size_t scratch_fock_offset(int ne, int nw) {
    return scratch_tag_offset(ne) + al16((size_t)(nw + 2) * 8);
}
__host__ __device__ inline size_t scratch_layout_bytes(int ne, int nw, int64_t n_fock) {
    return scratch_fock_offset(ne, nw) + (size_t)n_fock * 8;
}

// misc int slots
enum { MI_ST = 0, MI_PIV, MI_PTYPE, MI_PP, MI_PQ, MI_PA, MI_PB, MI_FS, MI_FW, MI_FK, MI_FFB, MI_SDNOW, MI_FTAG, MI_WAVE = 32 };
enum { MD_T = 0, MD_BASE, MD_EL, MD_HNN, MD_TARGET, MD_C00, MD_C01, MD_C10, MD_C11 };
// per-wave state: entries of the two batch logs and the stream ranges
enum { WS_NS = 0, WS_R1S = 3, WS_ND = 4, WS_R1D = 7 };

// 16x16x4 matrix-core step in the precision of R.  Operands: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; element j of the accumulator of lane
// l is D[row(l / 16, j)][l % 16] (the FP32 and FP64 instructions order the
// rows differently).
template <typename RT>
struct Mma;
template <>
struct Mma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int kq, int j) { return 4 * kq + j; }
};
template <>
struct Mma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int kq, int j) { return kq + 4 * j; }
};

// Split storage of the mixed form with the walker state in HBM: an R entry is
// hi + lo, hi its FP32 rounding and lo the bfloat16 rounding of the remainder
// (about 2^-33 relative in all).  The ratios read hi only; the re-inversion
// and every update carry both, so hi stays the rounding of the FP64 R instead
// of accumulating one FP32 rounding per move.
__device__ __forceinline__ uint16_t bf16_rn(float x) {
    return __builtin_bit_cast(uint16_t, (__bf16)x);  // v_cvt_pk_bf16_f32: round to nearest even
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ void store_split(float* hi, uint16_t* lo, size_t i, double v) {
    const float h = (float)v;
    hi[i] = h;
    lo[i] = (fabsf(h) <= FLT_MAX) ? bf16_rn((float)(v - (double)h)) : (uint16_t)0;
}

// R[p][a] = sum_x B[p][x] theta[a][x] (p < Ne slots, a < n_so orbitals, x < Ne)
// on the matrix cores: 16x16 output tiles dealt round-robin to the waves.
// Without SPLIT the operands are rounded to the precision of R and accumulated
// in it; with SPLIT (FP32 R with its bfloat16 remainder in Rlo) the product is
// formed in FP64 and stored split.
// th: theta[:, 0:Ne] with row stride ths (the table, or a copy in LDS).
template <typename RT, bool SPLIT = false>
__device__ __forceinline__ void r_gemm(const Tab& T, const double* B, RT* R, const double* th, int ths,
                                       uint16_t* Rlo = nullptr) {
    typedef typename std::conditional<SPLIT, double, RT>::type CT;
    const int ne = T.ne, n_so = T.n_so, l = lane_id();
    const int wv = (int)__builtin_amdgcn_readfirstlane((uint32_t)(threadIdx.x >> 6)), nwv = blockDim.x >> 6;
    const int mt = (ne + 15) >> 4, nt16 = (n_so + 15) >> 4;
    const int m = l & 15, kq = l >> 4;
    for (int t = wv; t < mt * nt16; t += nwv) {
        const int pt = t / nt16, at = t - pt * nt16;
        const int p = pt * 16 + m, a = at * 16 + m;
        typename Mma<CT>::acc_t acc = {0, 0, 0, 0};
#pragma unroll 4
        for (int k0 = 0; k0 < ne; k0 += 4) {
            const int x = k0 + kq;
            const CT av = (p < ne && x < ne) ? (CT)B[p * ne + x] : (CT)0;
            const CT bv = (a < n_so && x < ne) ? (CT)th[(size_t)a * ths + x] : (CT)0;
            acc = Mma<CT>::step(av, bv, acc);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int pr = pt * 16 + Mma<CT>::row(kq, j);
            if (pr < ne && a < n_so) {
                if constexpr (SPLIT) store_split(R, Rlo, (size_t)pr * n_so + a, acc[j]);
                else R[pr * n_so + a] = acc[j];
            }
        }
    }
}

// The same product with each wave holding a 16-orbital tile of theta in
// registers (KS k-steps, Ne <= 4 KS) across all slot tiles, so that theta is
// read once per walker instead of once per output tile; B in LDS.
template <typename RT, int KS, bool SPLIT = false>
__device__ __forceinline__ void r_gemm_theta_regs(const Tab& T, const double* B, RT* R, const double* th, int ths,
                                                  uint16_t* Rlo = nullptr) {
    typedef typename std::conditional<SPLIT, double, RT>::type CT;
    const int ne = T.ne, n_so = T.n_so, l = lane_id();
    const int wv = (int)__builtin_amdgcn_readfirstlane((uint32_t)(threadIdx.x >> 6)), nwv = blockDim.x >> 6;
    const int mt = (ne + 15) >> 4, nt16 = (n_so + 15) >> 4;
    const int m = l & 15, kq = l >> 4;
    for (int at = wv; at < nt16; at += nwv) {
        const int a = at * 16 + m;
        CT tr[KS];
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            const int x = 4 * st + kq;
            tr[st] = (a < n_so && x < ne) ? (CT)th[(size_t)a * ths + x] : (CT)0;
        }
        for (int pt = 0; pt < mt; ++pt) {
            const int p = pt * 16 + m;
            typename Mma<CT>::acc_t acc = {0, 0, 0, 0};
#pragma unroll
            for (int st = 0; st < KS; ++st)
                if (4 * st < ne) {
                    const int x = 4 * st + kq;
                    const CT av = (p < ne && x < ne) ? (CT)B[p * ne + x] : (CT)0;
                    acc = Mma<CT>::step(av, tr[st], acc);
                }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int pr = pt * 16 + Mma<CT>::row(kq, j);
                if (pr < ne && a < n_so) {
                    if constexpr (SPLIT) store_split(R, Rlo, (size_t)pr * n_so + a, acc[j]);
                    else R[pr * n_so + a] = acc[j];
                }
            }
        }
    }
}

// Row and column of the vector index vi = r * cv + c, stepped by a fixed
// stride with one division at set-up instead of one per step.
struct VecCursor {
    int r, c, dr, dc, cv;
    __device__ __forceinline__ VecCursor(int vi, int stride, int cv_) : cv(cv_) {
        r = vi / cv_;
        c = vi - r * cv_;
        dr = stride / cv_;
        dc = stride - dr * cv_;
    }
    __device__ __forceinline__ void advance() {
        r += dr;
        c += dc;
        if (c >= cv) {
            c -= cv;
            ++r;
        }
    }
};

// M[r][c] -= c1[c] r1[r] (+ c2[c] r2[r]) over rows x cols, by the whole block,
// arithmetic in FP64.  Rows are contiguous; when they split into 16-byte
// vectors each thread keeps four vector loads in flight (the update is a
// stream over HBM when the state does not fit on chip).
template <typename E, bool TWO>
__device__ __forceinline__ void rank_update(E* M, int rows, int cols, const double* c1, const double* r1,
                                            const double* c2, const double* r2) {
    constexpr int V = 16 / (int)sizeof(E);
    constexpr int U = 4;
    const int tid = threadIdx.x, nt = blockDim.x;
    struct alignas(16) Vec {
        E v[V];
    };
    if ((cols % V) == 0 && (((uintptr_t)M) & 15) == 0) {
        const int cv = cols / V, nv = rows * cv;
        Vec* Mv = (Vec*)M;
        VecCursor cur(tid, nt, cv);
        for (int v0 = tid; v0 < nv; v0 += nt * U) {
            Vec val[U];
            int rr[U], cc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int vi = v0 + u * nt;
                rr[u] = cur.r;
                cc[u] = cur.c * V;
                cur.advance();
                if (vi < nv) val[u] = Mv[vi];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int vi = v0 + u * nt;
                if (vi < nv) {
                    const int r = rr[u], c = cc[u];
                    const double a1 = r1[r], a2 = TWO ? r2[r] : 0.0;
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        double d = c1[c + j] * a1;
                        if (TWO) d += c2[c + j] * a2;
                        val[u].v[j] = (E)((double)val[u].v[j] - d);
                    }
                    Mv[vi] = val[u];
                }
            }
        }
    } else {
        for (int idx = tid; idx < rows * cols; idx += nt) {
            const int r = idx / cols, c = idx - r * cols;
            double d = c1[c] * r1[r];
            if (TWO) d += c2[c] * r2[r];
            M[idx] = (E)((double)M[idx] - d);
        }
    }
}

// The same on split storage (FP32 hi, bfloat16 lo): each entry is read as
// hi + lo, updated in FP64 and stored split again.  Vectors of four entries
// (16 bytes of hi, 8 of lo), four in flight per thread.
template <bool TWO>
__device__ __forceinline__ void rank_update_split(float* M, uint16_t* L, int rows, int cols, const double* c1,
                                                  const double* r1, const double* c2, const double* r2) {
    constexpr int U = 2;
    const int tid = threadIdx.x, nt = blockDim.x;
    struct alignas(16) V4 {
        float v[4];
    };
    struct alignas(8) L4 {
        uint16_t v[4];
    };
    if ((cols & 3) == 0 && (((uintptr_t)M) & 15) == 0 && (((uintptr_t)L) & 7) == 0) {
        const int cv = cols >> 2, nv = rows * cv;
        V4* Mv = (V4*)M;
        L4* Lv = (L4*)L;
        for (int v0 = tid; v0 < nv; v0 += nt * U) {
            V4 hv[U];
            L4 lv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int vi = v0 + u * nt;
                if (vi < nv) {
                    hv[u] = Mv[vi];
                    lv[u] = Lv[vi];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int vi = v0 + u * nt;
                if (vi < nv) {
                    const int r = vi / cv, c = (vi - r * cv) * 4;
                    const double a1 = r1[r], a2 = TWO ? r2[r] : 0.0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        double d = c1[c + j] * a1;
                        if (TWO) d += c2[c + j] * a2;
                        const double v = ((double)hv[u].v[j] + (double)bf16_val(lv[u].v[j])) - d;
                        const float h = (float)v;
                        hv[u].v[j] = h;
                        lv[u].v[j] = (fabsf(h) <= FLT_MAX) ? bf16_rn((float)(v - (double)h)) : (uint16_t)0;
                    }
                    Mv[vi] = hv[u];
                    Lv[vi] = lv[u];
                }
            }
        }
    } else {
        for (int idx = tid; idx < rows * cols; idx += nt) {
            const int r = idx / cols, c = idx - r * cols;
            double d = c1[c] * r1[r];
            if (TWO) d += c2[c] * r2[r];
            store_split(M, L, idx, ((double)M[idx] + (double)bf16_val(L[idx])) - d);
        }
    }
}

// Rank-1/2 update of R in its storage: split (mixed form, state in HBM) or plain.
template <typename RT, bool TWO, bool SPLIT>
__device__ __forceinline__ void r_update(RT* R, uint16_t* Rlo, int rows, int cols, const double* c1, const double* r1,
                                         const double* c2, const double* r2) {
    if constexpr (SPLIT) rank_update_split<TWO>(R, Rlo, rows, cols, c1, r1, c2, r2);
    else rank_update<RT, TWO>(R, rows, cols, c1, r1, c2, r2);
}

// The same on a sub-block whose rows lie ld elements apart (one spin's block
// of B with spin-blocked orbitals).
template <bool TWO>
__device__ __forceinline__ void rank_update_ld(double* M, int rows, int cols, int ld, const double* c1,
                                               const double* r1, const double* c2, const double* r2) {
    constexpr int U = 4;
    const int tid = threadIdx.x, nt = blockDim.x;
    if ((cols & 1) == 0 && (ld & 1) == 0 && (((uintptr_t)M) & 15) == 0) {
        // 16-byte vectors, four loads in flight per thread as in rank_update
        const int cv = cols >> 1, nv = rows * cv;
        VecCursor cur(tid, nt, cv);
        for (int v0 = tid; v0 < nv; v0 += nt * U) {
            double2 val[U];
            int rr[U], cc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int vi = v0 + u * nt;
                rr[u] = cur.r;
                cc[u] = cur.c * 2;
                cur.advance();
                if (vi < nv) val[u] = *(const double2*)(M + (size_t)rr[u] * ld + cc[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int vi = v0 + u * nt;
                if (vi < nv) {
                    const int r = rr[u], c = cc[u];
                    const double a1 = r1[r], a2 = TWO ? r2[r] : 0.0;
                    double d0 = c1[c] * a1, d1 = c1[c + 1] * a1;
                    if (TWO) {
                        d0 += c2[c] * a2;
                        d1 += c2[c + 1] * a2;
                    }
                    val[u].x -= d0;
                    val[u].y -= d1;
                    *(double2*)(M + (size_t)r * ld + c) = val[u];
                }
            }
        }
    } else {
        for (int idx = tid; idx < rows * cols; idx += nt) {
            const int r = idx / cols, c = idx - r * cols;
            double d = c1[c] * r1[r];
            if (TWO) d += c2[c] * r2[r];
            M[(size_t)r * ld + c] -= d;
        }
    }
}

// Rebuild B = theta[N]^-1 (Gauss-Jordan, partial pivoting, FP64), R and s from
// the slot list.  B is stored column by slot (B[x][p] at B[p*ne + x]): the
// elimination works on A^T, whose inverse laid out row-major is exactly that.
template <typename RT, bool SPLIT = false>
__device__ __forceinline__ void refresh_state(const Tab& T, const int* slot, double* B, RT* R, double* s, double* fcol, int* ipiv,
                              int* mi, double* red, const double* th, int ths, uint16_t* Rlo = nullptr) {
    const int tid = threadIdx.x, nt = blockDim.x, ne = T.ne, n_so = T.n_so;
    const int wv = tid >> 6, nwv = nt >> 6;
    for (int idx = tid; idx < ne * ne; idx += nt) {
        const int x = idx / ne, p = idx - x * ne;
        B[idx] = T.theta[(size_t)slot[p] * n_so + x];
    }
    __syncthreads();
    for (int k = 0; k < ne; ++k) {
        // every candidate starts at a valid row (k), and a NaN or infinite
        // entry ranks as the largest, so the pivot is always an unused row
        // below ne whatever the matrix holds; such a walker is flagged below
        double bv = -1.0;
        int bi = k;
        for (int r = k + tid; r < ne; r += nt) {
            double v = fabs(B[r * ne + k]);
            if (!(v <= DBL_MAX)) v = INFINITY;
            if (v > bv) { bv = v; bi = r; }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const double ov = __shfl_xor(bv, d, kWave);
            const int oi = __shfl_xor(bi, d, kWave);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane_id() == 0) { red[wv] = bv; mi[MI_WAVE + wv] = bi; }
        __syncthreads();
        if (tid == 0) {
            double best = red[0];
            int bidx = mi[MI_WAVE];
            for (int q = 1; q < nwv; ++q)
                if (red[q] > best || (red[q] == best && mi[MI_WAVE + q] < bidx)) { best = red[q]; bidx = mi[MI_WAVE + q]; }
            mi[MI_PIV] = bidx;
            ipiv[k] = bidx;
            if (!(best > 0.0)) mi[MI_ST] |= (int)VMC_ST_SINGULAR;
            if (!(best <= DBL_MAX)) mi[MI_ST] |= (int)(VMC_ST_SINGULAR | VMC_ST_NONFINITE);
        }
        __syncthreads();
        const int piv = mi[MI_PIV];
        if (piv != k)
            for (int c = tid; c < ne; c += nt) {
                const double t0 = B[k * ne + c];
                B[k * ne + c] = B[piv * ne + c];
                B[piv * ne + c] = t0;
            }
        __syncthreads();
        const double pv = B[k * ne + k];
        const double inv = (pv != 0.0) ? 1.0 / pv : 0.0;
        for (int r = tid; r < ne; r += nt) fcol[r] = B[r * ne + k];
        __syncthreads();
        for (int c = tid; c < ne; c += nt) B[k * ne + c] = (c == k) ? inv : B[k * ne + c] * inv;
        __syncthreads();
        for (int idx = tid; idx < ne * ne; idx += nt) {
            const int r = idx / ne, c = idx - r * ne;
            if (r == k) continue;
            B[idx] = (c == k) ? -fcol[r] * inv : B[idx] - fcol[r] * B[k * ne + c];
        }
        __syncthreads();
    }
    for (int k = ne - 1; k >= 0; --k) {
        const int piv = ipiv[k];
        if (piv != k)
            for (int r = tid; r < ne; r += nt) {
                const double t0 = B[r * ne + k];
                B[r * ne + k] = B[r * ne + piv];
                B[r * ne + piv] = t0;
            }
        __syncthreads();
    }
    r_gemm<RT, SPLIT>(T, B, R, th, ths, Rlo);
    for (int pp = tid; pp < n_so; pp += nt) {
        const double* Jr = T.J + (size_t)pp * n_so;
        double acc = 0.0;
        for (int k = 0; k < ne; ++k) {
            const int q = slot[k];
            if (q != pp) acc += Jr[q];
        }
        s[pp] = acc;
    }
    __syncthreads();
}


// In-place inclusive prefix sum of a[0..n) (u32) by the whole block; returns
// the total.  tmp: blockDim.x + 1 u32 of LDS.
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t* a, int n, uint32_t* tmp) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int chunk = (n + nt - 1) / nt;
    const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
    uint32_t sum = 0;
    for (int k = lo; k < hi; ++k) sum += a[k];
    tmp[tid] = sum;
    __syncthreads();
    if (tid < kWave) {
        uint32_t carry = 0;
        for (int base = 0; base < nt; base += kWave) {
            const int k = base + tid;
            const uint32_t v = (k < nt) ? tmp[k] : 0u;
            uint32_t x = v;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t y = __shfl_up(x, d, kWave);
                if (tid >= d) x += y;
            }
            if (k < nt) tmp[k] = carry + x - v;  // exclusive
            carry += __shfl(x, kWave - 1, kWave);
        }
        if (tid == 0) tmp[nt] = carry;
    }
    __syncthreads();
    uint32_t run = tmp[tid];
    for (int k = lo; k < hi; ++k) {
        run += a[k];
        a[k] = run;
    }
    const uint32_t total = tmp[nt];
    __syncthreads();
    return total;
}

// first group g with gend[g] > pos (gend inclusive-scanned, pos < gend[ng-1])
__device__ __forceinline__ uint32_t find_group(const uint32_t* gend, uint32_t ng, uint32_t pos) {
    uint32_t lo = 0, hi = ng - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (gend[mid] > pos) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Inclusive prefix sum of u32 over the wave (lane order).
__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t x) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, d, kWave);
        if (l >= d) x += y;
    }
    return x;
}

// Data-parallel-primitive move of a double (both halves), reading 0 where the
// row mask disables the destination.  With every row enabled each lane is
// written, so no zero needs to be placed in the destination first.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_d(double x) {
    int lo, hi;
    if constexpr (ROW_MASK == 0xF) {
        lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
        hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xF, false);
        hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xF, false);
    }
    return __hiloint2double(hi, lo);
}
// Sum over the 64 lanes in a fixed order (quads, rows of 16, then row
// broadcasts), returned as a wave-uniform value.
__device__ __forceinline__ double wave_total(double x) {
    x += dpp_d<0xB1>(x);        // quad_perm [1,0,3,2]
    x += dpp_d<0x4E>(x);        // quad_perm [2,3,0,1]
    x += dpp_d<0x124>(x);       // row_ror:4
    x += dpp_d<0x128>(x);       // row_ror:8
    x += dpp_d<0x142, 0xA>(x);  // row_bcast:15 into rows 1, 3
    x += dpp_d<0x143, 0xC>(x);  // row_bcast:31 into rows 2, 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), 63);
    return __hiloint2double(hi, lo);
}

// Largest u64 over the 64 lanes (same lane pattern as wave_total), returned
// as a wave-uniform value.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROW_MASK, 0xF, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
    x = umax64(x, dpp_u64<0xB1>(x));
    x = umax64(x, dpp_u64<0x4E>(x));
    x = umax64(x, dpp_u64<0x124>(x));
    x = umax64(x, dpp_u64<0x128>(x));
    x = umax64(x, dpp_u64<0x142, 0xA>(x));
    x = umax64(x, dpp_u64<0x143, 0xC>(x));
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

// Block-wide deterministic sum (every thread gets the same value).
__device__ __forceinline__ double block_total(double v, double* red) {
    const int wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    v = wave_total(v);
    if (lane_id() == 0) red[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < nwv; ++k) t += red[k];
    __syncthreads();
    return t;
}

// One walker's per-step data.  The candidate stream of each kind is the
// concatenation of its groups' table rows (singles: one group per occupied
// orbital; doubles: one per occupied pair), each padded to a multiple of 64
// positions so that a 64-lane chunk lies within one group.  With the walker
// state in HBM the singles rows are not padded (see stream_pass).
template <typename RT>
struct StepView {
    const int* occl;
    const double* es;     // exp(s_p)          (unscaled path)
    const RT* R;          // R (unscaled path) or Rh[p][a] = R[a][p] exp(s_a - s_orb(p)) (scaled path)
    const uint32_t* sgend;  // singles: padded inclusive stream ends per occupied index
    const uint32_t* sdelta; //          table offset = stream position + delta
    const uint32_t* svend;  //          end of the group's valid positions
    const uint32_t* spq;    //          slot of the occupied orbital
    const double* sfac;     //          exp(-s_i) (unscaled path)
    const uint32_t* dgend;  // doubles: the same per occupied pair
    const uint32_t* ddelta;
    const uint32_t* dvend;
    const uint32_t* dpq;    //          slots p | q << 16
    const double* ies;      // exp(-s_p)         (unscaled path)
    const int* slot;        // orbital held by each slot
    const uint32_t* cidx;   // correlators: current local Fock state of each
    const double* cinv;     //              and 1 / its coefficient
    const double* F;        // singles elements h_ia + sum_{j occupied} V_ia[j] per table entry (state in
                            // HBM with Coulomb-exchange vectors), else null
    const double* sies;     // exp(-s) of the orbital each slot holds (unscaled path)
};

// Fock-like singles elements F[e] = h_ia + sum_{j occupied} V_e[j] (the
// element of the section "Reduced scaling evaluation of the local energy"
// before its phase) for every entry e of the rows of the orbitals rows[0..nr),
// from scratch over the occupied orbitals occ[0..ne): one wave per row, lanes
// over its entries (the j-major vectors make them contiguous for each j).
__device__ __forceinline__ void fock_rows(const Tab& T, double* F, const int* rows, int nr, const int* occ, int ne) {
    const int l = lane_id(), wv = (int)uni((uint32_t)(threadIdx.x >> 6)), nwv = blockDim.x >> 6;
    for (int x = wv; x < nr; x += nwv) {
        const int r = rows[x];
        const uint32_t b0 = T.s_off[r], len = T.s_off[r + 1] - b0;
        for (uint32_t e = l; e < len; e += kWave) {
            const double* Vr = T.sV + (size_t)b0 * T.n_so + e;
            double h = T.sh[b0 + e];
#pragma unroll 8
            for (int y = 0; y < ne; ++y) h += Vr[(size_t)occ[y] * len];
            F[b0 + e] = h;
        }
    }
}

// After a move that empties i (j) and fills a (b): the rows of the orbitals
// occupied before and after change by V_e[a] - V_e[i] (+ V_e[b] - V_e[j]);
// the rows of a (b) are built from scratch over the new occupation slot[0..ne).
__device__ __forceinline__ void fock_move(const Tab& T, double* F, const int* slot, int ne, int i, int j, int a, int b) {
    const int l = lane_id(), wv = (int)uni((uint32_t)(threadIdx.x >> 6)), nwv = blockDim.x >> 6;
    for (int x = wv; x < ne; x += nwv) {
        const int r = slot[x];
        const uint32_t b0 = T.s_off[r], len = T.s_off[r + 1] - b0;
        const bool fresh = (r == a) || (b >= 0 && r == b);
        for (uint32_t e = l; e < len; e += kWave) {
            const double* Vr = T.sV + (size_t)b0 * T.n_so + e;
            if (fresh) {
                double h = T.sh[b0 + e];
#pragma unroll 8
                for (int y = 0; y < ne; ++y) h += Vr[(size_t)slot[y] * len];
                F[b0 + e] = h;
            } else {
                double d = Vr[(size_t)a * len] - Vr[(size_t)i * len];
                if (b >= 0) d += Vr[(size_t)b * len] - Vr[(size_t)j * len];
                F[b0 + e] += d;
            }
        }
    }
}

// Correlator ratio C[M]/C[N] (section "Local energy and Gradient ratios": only
// the correlators holding a site whose occupation changes enter, each once).
// The move empties the first nk/2 orbitals o0 (o1) and fills the other nk/2
// (nk = 2: i -> a; nk = 4: i, j -> a, b).  For each correlator holding the
// site of some changed orbital, its state in M is its state in N plus, for
// every changed orbital on its sites, -1 (emptied) or +1 (filled) times the
// orbital's digit weight (1 alpha, 2 beta) times 4^(position of the site);
// the ratio multiplies c[state in M] / c[state in N].  Inlined: a call would
// make the sweep kernels, whose register budget is fixed by their occupancy
// target, save their live registers to scratch around it.
__device__ __forceinline__ double cps_ratio(const Tab& T, const uint32_t* cidx, const double* cinv, int nk, int o0,
                                            int o1, int o2, int o3) {
    const int n = T.n;
    int st[4], wt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int o = k == 0 ? o0 : k == 1 ? o1 : k == 2 ? o2 : o3;
        st[k] = (k < nk) ? ((o >= n) ? o - n : o) : -2;
        wt[k] = ((k < nk / 2) ? -1 : 1) * ((o >= n) ? 2 : 1);
    }
    double r = 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k >= nk) break;
        const int e1 = T.sc_off[st[k] + 1];
        for (int e = T.sc_off[st[k]]; e < e1; ++e) {
            const int lam = (int)(T.sc_list[e] & 0xFFFFFFu);
            const int* cs = T.csite + 5 * lam;
            const int c0 = cs[0], c1 = cs[1], c2 = cs[2], c3 = cs[3], c4 = cs[4];
            auto pos = [&](int x) {
                return x == c0 ? 0 : x == c1 ? 1 : x == c2 ? 2 : x == c3 ? 3 : x == c4 ? 4 : -1;
            };
            bool seen = false;
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2)
                if (k2 < k) seen = seen || pos(st[k2]) >= 0;
            if (seen) continue;  // handled with the earlier orbital's correlators
            int delta = 0;
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) {
                const int m = (k2 < nk) ? pos(st[k2]) : -1;
                if (m >= 0) delta += wt[k2] * (1 << (2 * m));
            }
            r *= T.cc[T.coff[lam] + (int)cidx[lam] + delta] * cinv[lam];
        }
    }
    return r;
}

// Local Fock state of every correlator in the occupation occw, and the inverse
// of its coefficient, by the whole block (LDS outputs).
__device__ __forceinline__ void cps_states(const Tab& T, const uint64_t* occw, uint32_t* cidx, double* cinv) {
    for (int lam = threadIdx.x; lam < T.ncorr; lam += blockDim.x) {
        uint32_t idx = 0, w = 1;
        for (int m = 0; m < 5; ++m) {
            const int site = T.csite[5 * lam + m];
            if (site < 0) break;
            const int b = site + T.n;
            idx += w * (uint32_t)(((occw[site >> 6] >> (site & 63)) & 1ull) + 2 * ((occw[b >> 6] >> (b & 63)) & 1ull));
            w *= 4;
        }
        cidx[lam] = idx;
        cinv[lam] = 1.0 / T.cc[T.coff[lam] + (int)idx];
    }
}

// Ratio psi(M)/psi(N) (and, when WANT_H, the local-energy term H_NM * ratio)
// of a queued candidate: table offset `off`, group g, targets in `ab` (a
// 64-bit occupancy mask when MASK, else a | b << 16 / a in the low word).
// Unscaled without MASK (group descriptors in HBM), the high word of `ab`
// carries the group's slots p | q << 16 / p, so the R loads need no
// descriptor load first.
template <bool DOUBLES, bool WANT_H, bool MASK, bool SCALED, bool UHF, typename RT>
__device__ __forceinline__ double cand_eval(const Tab& T, const StepView<RT>& V, uint32_t off, uint32_t g, uint64_t ab,
                                            double2 vk, double& term, int& cp, int& cq, int& ca, int& cb) {
    constexpr bool QPQ = !SCALED && !MASK;
    const int n_so = T.n_so;
    if (DOUBLES) {
        const uint32_t pq = QPQ ? (uint32_t)(ab >> 32) : V.dpq[g];
        const int p = (int)(pq & 0xFFFFu), q = (int)(pq >> 16);
        int a, b;
        if (MASK) {
            a = __builtin_ctzll(ab);
            b = 63 - __builtin_clzll(ab);
        } else {
            a = (int)(ab & 0xFFFFu);
            b = (int)((ab >> 16) & 0xFFFFu);
        }
        double det;
        if (UHF) {
            det = pair_minor_uhf(T, V.R, p, q, a, b);
        } else {
            const RT* Rp = V.R + __umul24((uint32_t)p, (uint32_t)n_so);
            const RT* Rq = V.R + __umul24((uint32_t)q, (uint32_t)n_so);
            if constexpr (sizeof(RT) == 8) det = minor_of(Rp[a], Rq[b], Rp[b], Rq[a]);
            else det = (double)Rp[a] * (double)Rq[b] - (double)Rp[b] * (double)Rq[a];
        }
        double ratio = SCALED ? det * vk.y : det * V.es[a] * V.es[b] * vk.y * (V.sies[p] * V.sies[q]);
        if (T.ncorr) ratio *= cps_ratio(T, V.cidx, V.cinv, 4, V.slot[p], V.slot[q], a, b);
        if (WANT_H) term = vk.x * ratio;
        cp = p; cq = q; ca = a; cb = b;
        return ratio;
    } else {
        const int p = QPQ ? (int)(ab >> 32) : (int)V.spq[g];
        const int a = (int)(uint32_t)ab;
        const double r1 = (double)V.R[UHF ? r_index_uhf(T, p, a) : p * n_so + a];
        double ratio = SCALED ? r1 * T.sK[off] : r1 * V.es[a] * V.sfac[g] * T.sK[off];
        if (T.ncorr) ratio *= cps_ratio(T, V.cidx, V.cinv, 2, V.slot[p], a, 0, 0);
        if (WANT_H && V.F) {
            term = V.F[off] * ratio;
        } else if (WANT_H) {
            double h = T.sh[off];
            if (T.has_sV) {
                // the row of orbital i stores V[j] of its entries contiguously
                // for each j, so the lanes of one group read together
                const int i = V.occl[g];
                const uint32_t b0 = T.s_off[i], len = T.s_off[i + 1] - b0;
                const double* Vr = T.sV + (size_t)b0 * n_so + (off - b0);
#pragma unroll 4
                for (int y = 0; y < T.ne; ++y) h += Vr[(size_t)V.occl[y] * len];
            }
            term = h * ratio;
        }
        cp = p; cq = -1; ca = a; cb = -1;
        return ratio;
    }
}

// Batch log of one wave (wave-uniform bookkeeping).  The candidate stream is
// cut into entries of `gran` consecutive 64-candidate batches; an entry keeps
// its rate sum and the table offset / group of its first candidate.  Rates of
// the open entry accumulate per lane and are reduced once when it closes.  A
// full log merges neighbouring entries pairwise and doubles `gran`.
struct BatchLog {
    double* sum;
    uint32_t* off;
    uint32_t* grp;
    int cap, n, gran, cnt;
    uint32_t cur_off, cur_g;
    double acc;
    __device__ __forceinline__ void add_batch(double r, uint32_t o0, uint32_t g0) {
        if (cnt == 0) { cur_off = o0; cur_g = g0; acc = 0.0; }
        acc += r;
        if (++cnt == gran) close();
    }
    __device__ __forceinline__ void close() {
        if (cnt == 0) return;
        const double s = wave_total(acc);
        const int l = lane_id();
        if (n == cap) {
            wave_lds_sync();
            double a0 = 0.0, a1 = 0.0;
            uint32_t oo = 0, gg = 0;
            const int half = cap >> 1;
            if (l < half) { a0 = sum[2 * l]; a1 = sum[2 * l + 1]; oo = off[2 * l]; gg = grp[2 * l]; }
            wave_lds_sync();
            if (l < half) { sum[l] = a0 + a1; off[l] = oo; grp[l] = gg; }
            wave_lds_sync();
            n = half;
            gran *= 2;
        }
        if (l == 0) { sum[n] = s; off[n] = cur_off; grp[n] = cur_g; }
        ++n;
        cnt = 0;
    }
};

// Pass over the padded stream chunks [c0, c1) of one wave (multiples of 64);
// g0 = group of c0; positions below `first` are skipped.
// ELOC: accumulate local-energy terms in `el`, log rate sums.
// PICK: with running sum `base` at `first`, find the candidate where the
// running sum first exceeds `target` (or, with `fallback` or after rounding,
// the last positive-rate candidate); pick = {type, p, q, a, b}; returns true
// if found.
// The table loads of kUnroll chunks are issued together before they are consumed.
template <bool DOUBLES, bool PICK, bool NW1, bool SCALED, bool UHF, typename RT>
__device__ __forceinline__ bool stream_pass(const Tab& T, const StepView<RT>& V, uint64_t occ0, const uint64_t* occw, uint32_t c0,
                            uint32_t c1, uint32_t g0, uint32_t ng, uint32_t first, uint64_t* q64, uint64_t* qab,
                            double& el, double* log_sum, uint32_t* log_off, uint32_t* log_grp, int log_cap, int& log_n,
                            double base, double target, bool fallback, int* pick) {
    BatchLog lg{log_sum, log_off, log_grp, log_cap, 0, kLogGran, 0, 0u, 0u, 0.0};
    BatchLog* log = &lg;
    // Survival test of a doubles entry: with one occupancy word, one AND of
    // the entry's target-orbital mask; otherwise two occupancy bit tests.
    constexpr bool MASK = DOUBLES && NW1;
    const int l = lane_id();
    c0 = uni(c0);
    c1 = uni(c1);
    first = uni(first);
    const uint32_t* gend = DOUBLES ? V.dgend : V.sgend;
    const uint32_t* delta = DOUBLES ? V.ddelta : V.sdelta;
    const uint32_t* vend = DOUBLES ? V.dvend : V.svend;
    // Group cursor.  Descriptors in LDS: scalar, advanced group by group.
    // Descriptors in HBM (unscaled variant): a block of 64 consecutive groups
    // held one per lane, the chunk's group found by a ballot, so that empty
    // groups cost nothing and descriptor loads are coalesced.
    constexpr bool REG_CURSOR = !SCALED;
    // Singles with their descriptors in LDS and the walker state in HBM: the
    // groups are not padded (a Hubbard electron has only a few targets), so a
    // chunk may span several groups and each lane finds its own by a binary
    // search over the group ends, from a lower bound carried chunk to chunk.
    constexpr bool DENSE = !DOUBLES && REG_CURSOR;
    // queue entries carry the group's slots (see cand_eval)
    constexpr bool QPQ = REG_CURSOR && !MASK;
    const uint32_t* gpq = DOUBLES ? V.dpq : V.spq;
    // survivor queue: a ring of kQueue entries, head qh, qn entries queued
    uint32_t gc = uni(g0), qn = 0, qh = 0;
    uint32_t e_end = 0, e_vend = 0, e_delta = 0, e_pq = 0;
    uint32_t blk = 0, b_end = 0, b_vend = 0, b_delta = 0, b_pq = 0;
    auto load_block = [&]() __attribute__((always_inline)) {
        const uint32_t gg = blk + (uint32_t)l;
        const bool in = gg < ng;
        b_end = in ? gend[gg] : 0xFFFFFFFFu;
        b_vend = in ? vend[gg] : 0u;
        b_delta = in ? delta[gg] : 0u;
        if (QPQ) b_pq = in ? gpq[gg] : 0u;
    };
    if (DENSE) {
        // gc: a lower bound of the group of every position still to come
    } else if (REG_CURSOR) {
        blk = gc & ~63u;
        load_block();
    } else {
        e_end = uni(gend[gc]);
        e_vend = uni(vend[gc]);
        e_delta = uni(delta[gc]);
    }
    double run = base;
    bool found = false;
    int last_l = -1;
    uint32_t last_off = 0, last_g = 0;
    uint64_t last_ab = 0;

    struct Stage {
        uint32_t g[kUnroll], off[kUnroll], pq[kUnroll];
        bool ok[kUnroll];
        uint64_t ab[kUnroll];
    };
    // compute the chunks' groups and offsets (advancing the uniform group
    // cursor) and issue their table loads
    auto fetch = [&](uint32_t c, Stage& st) __attribute__((always_inline)) {
        uint32_t gnext = gc;  // dense singles: the searches of one fetch share gc as their lower bound
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint32_t cu = c + (uint32_t)(u * kWave);
            st.ok[u] = false;
            st.g[u] = gc;
            st.off[u] = 0;
            st.pq[u] = 0;
            if (DENSE && cu < c1) {
                const uint32_t pos = cu + (uint32_t)l;
                uint32_t lo = gc, hi = ng - 1;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (gend[mid] > pos) hi = mid;
                    else lo = mid + 1;
                }
                st.g[u] = lo;
                st.pq[u] = gpq[lo];
                st.ok[u] = pos < vend[lo] && pos >= first;
                st.off[u] = st.ok[u] ? pos + delta[lo] : 0u;  // entry 0 stands in for lanes without a candidate
                gnext = (uint32_t)__builtin_amdgcn_readlane((int)lo, kWave - 1);
            } else if (cu < c1) {
                if (REG_CURSOR) {
                    uint64_t m = __ballot(b_end > cu);
                    while (m == 0ull) {
                        blk += kWave;
                        load_block();
                        m = __ballot(b_end > cu);
                    }
                    const int gl = (int)__builtin_amdgcn_readfirstlane((uint32_t)(__ffsll((unsigned long long)m) - 1));
                    gc = blk + (uint32_t)gl;
                    e_vend = (uint32_t)__builtin_amdgcn_readlane((int)b_vend, gl);
                    e_delta = (uint32_t)__builtin_amdgcn_readlane((int)b_delta, gl);
                    if (QPQ) e_pq = (uint32_t)__builtin_amdgcn_readlane((int)b_pq, gl);
                } else {
                    while (e_end <= cu) {
                        ++gc;
                        e_end = uni(gend[gc]);
                        e_vend = uni(vend[gc]);
                        e_delta = uni(delta[gc]);
                    }
                }
                st.g[u] = gc;
                st.pq[u] = e_pq;
                const uint32_t pos = cu + (uint32_t)l;
                st.ok[u] = pos < e_vend && pos >= first;
                st.off[u] = st.ok[u] ? pos + e_delta : 0u;  // entry 0 stands in for lanes without a candidate
            }
        }
        if (DENSE) gc = gnext;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (MASK) st.ab[u] = T.dmask[st.off[u]];
            else if (DOUBLES) st.ab[u] = T.dab[st.off[u]];
            else st.ab[u] = T.sa[st.off[u]];
        }
    };
    auto batch = [&](int k) __attribute__((always_inline)) -> bool {
        wave_lds_sync();
        const bool act = l < k;
        const uint32_t qi = (qh + (uint32_t)l) & (kQueue - 1);
        const uint64_t og = act ? q64[qi] : 0ull;
        const uint32_t off = (uint32_t)og, g = (uint32_t)(og >> 32);
        const uint64_t ab = act ? qab[qi] : 0ull;
        double2 vk = make_double2(0.0, 0.0);
        if (DOUBLES && act) vk = *(const double2*)(T.dvK + 2 * (size_t)off);
        double term = 0.0, r = 0.0;
        int cp = 0, cq = 0, ca = 0, cb = 0;
        if (act) r = fabs(cand_eval<DOUBLES, !PICK, MASK, SCALED, UHF>(T, V, off, g, ab, vk, term, cp, cq, ca, cb));
        if (!PICK) {
            el += term;
            log->add_batch(r, uni((uint32_t)og), uni((uint32_t)(og >> 32)));
            return false;
        }
        const uint64_t mpos = __ballot(r > 0.0);
        if (mpos) {
            last_l = 63 - __clzll((long long)mpos);
            last_off = __shfl(off, last_l, kWave);
            last_g = __shfl(g, last_l, kWave);
            last_ab = ((uint64_t)__shfl((uint32_t)(ab >> 32), last_l, kWave) << 32) |
                      (uint64_t)__shfl((uint32_t)ab, last_l, kWave);
        }
        if (fallback) return false;
        const double incl = wave_inclusive_scan(r);
        const uint64_t mx = __ballot(act && r > 0.0 && run + incl > target);
        if (mx) {
            const int fl = __ffsll((unsigned long long)mx) - 1;
            if (l == fl) { pick[0] = DOUBLES ? 2 : 1; pick[1] = cp; pick[2] = cq; pick[3] = ca; pick[4] = cb; }
            return true;
        }
        run += __shfl(incl, kWave - 1, kWave);
        return false;
    };
    auto consume = [&](const Stage& st) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            bool surv;
            if (MASK) {
                surv = st.ok[u] && (st.ab[u] & occ0) == 0ull;
            } else if (DOUBLES) {
                const uint32_t a = (uint32_t)st.ab[u] & 0xFFFFu, b = (uint32_t)st.ab[u] >> 16;
                surv = st.ok[u] && !((occw[a >> 6] >> (a & 63)) & 1ull) && !((occw[b >> 6] >> (b & 63)) & 1ull);
            } else {
                const uint32_t a = (uint32_t)st.ab[u];
                surv = st.ok[u] && (NW1 ? !((occ0 >> a) & 1ull) : !((occw[a >> 6] >> (a & 63)) & 1ull));
            }
            surv = surv && !found;
            const uint64_t m = __ballot(surv);
            if (surv) {
                const uint32_t sq = (qh + qn + mask_below(m)) & (kQueue - 1);
                q64[sq] = (uint64_t)st.off[u] | ((uint64_t)st.g[u] << 32);
                qab[sq] = QPQ ? (st.ab[u] & 0xFFFFFFFFull) | ((uint64_t)st.pq[u] << 32) : st.ab[u];
            }
            qn += (uint32_t)__popcll(m);
            if (qn >= (uint32_t)kWave) {
                found = batch(kWave);
                wave_lds_sync();  // the batch's queue reads precede later writes
                qh = (qh + kWave) & (kQueue - 1);
                qn -= kWave;
            }
        }
    };
    for (uint32_t c = c0; c < c1 && !found; c += kUnroll * kWave) {
        Stage st;
        fetch(c, st);
        consume(st);
    }
    if (!found && qn > 0) found = batch((int)qn);
    if (!PICK) log->close();
    log_n = lg.n;
    wave_lds_sync();
    if (PICK && !found && last_l >= 0) {
        // rounding left the target past the last running sum: take the last
        // candidate with a positive rate
        if (l == 0) {
            double term;
            int cp, cq, ca, cb;
            const double2 vk = DOUBLES ? *(const double2*)(T.dvK + 2 * (size_t)last_off) : make_double2(0.0, 0.0);
            cand_eval<DOUBLES, false, MASK, SCALED, UHF>(T, V, last_off, last_g, last_ab, vk, term, cp, cq, ca, cb);
            pick[0] = DOUBLES ? 2 : 1; pick[1] = cp; pick[2] = cq; pick[3] = ca; pick[4] = cb;
        }
        found = true;
    }
    return found;
}

// Doubles of the layout with the walker state in HBM, over tiles of occupied
// pairs.  The occupied orbitals (ascending, index x) are cut into blocks of
// kPairBlock.  Segment (x, Y) is the run of pairs (x, y), y > x, y in block Y:
// a contiguous piece of the canonical order (pairs by x, then by y), whose
// rate sum goes to segsum[x * nb + Y].  Tiles (X, Y), X <= Y, are visited
// Y-major by all waves of the workgroup together (segment x of tile k to wave
// (x - X kPairBlock + k) mod nwv), so that the rows of R of the two blocks,
// which the pairs' 2x2 minors gather, are reused from the caches across the
// tile instead of fetched once per pair.  The lanes hold the table rows of
// kWave / kPairBlock of the wave's segments at a time (pair p of segment s
// in lane kPairBlock s + p, then the rows with entries moved to the lowest
// lanes); their entries form one unpadded stream, cut into 64-entry chunks, so that the table loads of
// several rows and segments go out together.  A lane finds its row in
// constant time: the rows starting inside the chunk set one marker byte each
// in LDS, and the lane counts the markers below it (one ballot, one mbcnt).
// An entry survives when both its target orbitals are empty (their slots are
// -1).  Survivors queue and are evaluated 64 at a time as in stream_pass; the
// queue keeps processing order, so each segment's survivors form one run of
// lanes.
// ELOC: E_L terms into `el`, rate sums per segment (segments without
// survivors keep the zero written before).  PICK: segment (px, py) only,
// running sum from `base`, pick as stream_pass.
template <bool PICK, bool UHF, typename RT>
__device__ __forceinline__ bool pair_tiles(const Tab& T, const StepView<RT>& V, const int* oslot, uint8_t* mark,
                                           uint64_t* q64, uint64_t* qab, double& el, double* segsum, int px, int py,
                                           double base, double target, bool fallback, int* pick) {
    constexpr int kSegs = kWave / kPairBlock;  // segments held by the lanes at once
    const int l = lane_id();
    const int wv = (int)uni((uint32_t)(threadIdx.x >> 6)), nwv = blockDim.x >> 6;
    const int ne = T.ne, n_so = T.n_so, nb = pair_blocks(ne);
    uint32_t qn = 0, qh = 0;
    double run = base;
    bool found = false;
    int last_l = -1;
    uint32_t last_off = 0;
    uint64_t last_ab = 0;
    // ELOC: the open segment (wave-uniform) and each lane's part of its rate
    // sum; a segment is reduced across the wave once, when the next one opens
    int cur_s = -1;
    double acc = 0.0;
    // the wave's marker bytes (kTileUnroll x 64) are zero between uses
    for (int k = l; k < kTileUnroll * kWave / 4; k += kWave) ((uint32_t*)mark)[k] = 0u;
    wave_lds_sync();

    auto batch = [&](int k) __attribute__((always_inline)) -> bool {
        wave_lds_sync();
        const bool act = l < k;
        const uint32_t qi = (qh + (uint32_t)l) & (kQueue - 1);
        const uint64_t og = act ? q64[qi] : 0ull;
        const uint32_t off = (uint32_t)og, sg = (uint32_t)(og >> 32);
        const uint64_t ab = act ? qab[qi] : 0ull;
        double term = 0.0, r = 0.0;
        int cp = 0, cq = 0, ca = 0, cb = 0;
        if (act) {
            const double2 vk = *(const double2*)(T.dvK + 2 * (size_t)off);
            r = fabs(cand_eval<true, !PICK, false, false, UHF>(T, V, off, 0u, ab, vk, term, cp, cq, ca, cb));
        }
        if (!PICK) {
            el += term;
            // the batch's lanes hold runs of segments in processing order: the
            // first run may continue the open segment; every later run opens
            // a new one, which closes the one before it
            const bool inc = act && (int)sg == cur_s;
            acc += inc ? r : 0.0;
            uint64_t rem = __ballot(act) & ~__ballot(inc);
            while (rem) {
                if (cur_s >= 0) {
                    const double tot = wave_total(acc);
                    if (l == 0) segsum[cur_s] = tot;
                }
                const int fl = __ffsll((unsigned long long)rem) - 1;
                const int s0 = __builtin_amdgcn_readlane((int)sg, fl);
                const bool in = act && (int)sg == s0;
                acc = in ? r : 0.0;
                cur_s = s0;
                rem &= ~__ballot(in);
            }
            return false;
        }
        const uint64_t mpos = __ballot(r > 0.0);
        if (mpos) {
            last_l = 63 - __clzll((long long)mpos);
            last_off = __shfl(off, last_l, kWave);
            last_ab = ((uint64_t)__shfl((uint32_t)(ab >> 32), last_l, kWave) << 32) |
                      (uint64_t)__shfl((uint32_t)ab, last_l, kWave);
        }
        if (fallback) return false;
        const double incl = wave_inclusive_scan(r);
        const uint64_t mx = __ballot(act && r > 0.0 && run + incl > target);
        if (mx) {
            const int fl = __ffsll((unsigned long long)mx) - 1;
            if (l == fl) { pick[0] = 2; pick[1] = cp; pick[2] = cq; pick[3] = ca; pick[4] = cb; }
            return true;
        }
        run += __shfl(incl, kWave - 1, kWave);
        return false;
    };

    // ELOC with FP64 R: a full batch's table and R loads are issued when it
    // fills and its terms formed when the next one fills (or at the end), so
    // that its gathers are in flight during the scan of the chunks that
    // follow.  Lanes without a candidate load entry 0 of both (spin-blocked:
    // a pair of opposite spins loads two entries).  (Measured: the FP64 sweep
    // 5.5 % faster at 160 orbitals and 6 % at 40; with FP32 R, whose gathers
    // take half the bytes, 1.4 % slower.)
    constexpr bool DEFER = !PICK && sizeof(RT) == 8;
    bool pend = false, p_act = false;
    uint32_t p_sg = 0;
    uint64_t p_ab = 0;
    double2 p_vk = make_double2(0.0, 0.0);
    RT p_x0 = 0, p_x1 = 0, p_x2 = 0, p_x3 = 0;
    auto issue = [&](int k) __attribute__((always_inline)) {
        wave_lds_sync();
        p_act = l < k;
        const uint32_t qi = (qh + (uint32_t)l) & (kQueue - 1);
        const uint64_t og = p_act ? q64[qi] : 0ull;
        p_ab = p_act ? qab[qi] : 0ull;
        p_sg = (uint32_t)(og >> 32);
        const uint32_t a = (uint32_t)p_ab & 0xFFFFu, b = (uint32_t)(p_ab >> 16) & 0xFFFFu;
        const uint32_t pp = (uint32_t)(p_ab >> 32) & 0xFFFFu, qq = (uint32_t)(p_ab >> 48);
        p_vk = *(const double2*)(T.dvK + 2 * (size_t)(uint32_t)og);
        if (UHF) {
            // (slot 0 of a lane without a candidate counts as alpha: row 0)
            const int op = (p_act && (int)pp >= T.na) ? T.n : 0, oq = (p_act && (int)qq >= T.na) ? T.n : 0;
            const RT* Rp = V.R + ((int)pp * T.n - op);
            const RT* Rq = V.R + ((int)qq * T.n - oq);
            p_x0 = Rp[a];
            p_x1 = Rq[b];
            p_x2 = (op == oq) ? Rp[b] : (RT)0;
            p_x3 = (op == oq) ? Rq[a] : (RT)0;
        } else {
            const RT* Rp = V.R + __umul24(pp, (uint32_t)n_so);
            const RT* Rq = V.R + __umul24(qq, (uint32_t)n_so);
            p_x0 = Rp[a]; p_x1 = Rq[b]; p_x2 = Rp[b]; p_x3 = Rq[a];
        }
        pend = true;
    };
    auto finish = [&]() __attribute__((always_inline)) {
        if (!pend) return;
        pend = false;
        double term = 0.0, r = 0.0;
        if (p_act) {
            const int a = (int)(p_ab & 0xFFFFu), b = (int)((p_ab >> 16) & 0xFFFFu);
            const int p = (int)((p_ab >> 32) & 0xFFFFu), q = (int)(p_ab >> 48);
            const bool opp = UHF && ((p >= T.na) != (q >= T.na));
            const double det = opp ? (double)p_x0 * (double)p_x1 : minor_of(p_x0, p_x1, p_x2, p_x3);
            double ratio = det * V.es[a] * V.es[b] * p_vk.y * (V.sies[p] * V.sies[q]);
            if (T.ncorr) ratio *= cps_ratio(T, V.cidx, V.cinv, 4, V.slot[p], V.slot[q], a, b);
            term = p_vk.x * ratio;
            r = fabs(ratio);
        }
        el += term;
        const bool inc = p_act && (int)p_sg == cur_s;
        acc += inc ? r : 0.0;
        uint64_t rem = __ballot(p_act) & ~__ballot(inc);
        while (rem) {
            if (cur_s >= 0) {
                const double tot = wave_total(acc);
                if (l == 0) segsum[cur_s] = tot;
            }
            const int fl = __ffsll((unsigned long long)rem) - 1;
            const int s0 = __builtin_amdgcn_readlane((int)p_sg, fl);
            const bool in = p_act && (int)p_sg == s0;
            acc = in ? r : 0.0;
            cur_s = s0;
            rem &= ~__ballot(in);
        }
    };

    // the wave's segments in order (wave-uniform): tiles Y-major, in tile k
    // the local rows xl = wv - k (mod nwv), xl + nwv, ...; empty segments skipped
    int it_yb = 0, it_xb = 0, it_k = 0, it_xl = wv % nwv;
    bool it_done = PICK;
    auto next_seg = [&](int& x, int& yb) __attribute__((always_inline)) -> bool {
        while (!it_done) {
            if (it_xl >= kPairBlock || it_xb * kPairBlock + it_xl >= ne - 1) {
                ++it_k;
                if (++it_xb > it_yb) {
                    it_xb = 0;
                    if (++it_yb >= nb) {
                        it_done = true;
                        break;
                    }
                }
                it_xl = (wv - it_k) % nwv;
                if (it_xl < 0) it_xl += nwv;
                continue;
            }
            x = it_xb * kPairBlock + it_xl;
            yb = it_yb;
            it_xl += nwv;
            if (max(x + 1, yb * kPairBlock) <= min(ne, (yb + 1) * kPairBlock) - 1) return true;
        }
        return false;
    };

    bool first = true;
    while (!found) {
        // the next (up to) four segments into the lanes
        int sx[kSegs], sy[kSegs], nseg = 0;
#pragma unroll
        for (int k = 0; k < kSegs; ++k) {
            sx[k] = 0;
            sy[k] = 0;
            if (PICK) {
                if (k == 0 && first) { sx[0] = px; sy[0] = py; nseg = 1; }
            } else if (nseg == k && next_seg(sx[k], sy[k])) {
                nseg = k + 1;
            }
        }
        first = false;
        if (nseg == 0) break;
        const int sl = l / kPairBlock, pl = l - sl * kPairBlock;
        int x = sx[0], yb = sy[0];
#pragma unroll
        for (int k = 1; k < kSegs; ++k)
            if (sl == k) { x = sx[k]; yb = sy[k]; }
        // lane (kPairBlock s + p): the table row of pair p of segment s, its slots
        // (16 bits each) and the segment's index
        uint32_t b0 = 0, len = 0, pk = 0, sg = 0;
        if (sl < nseg) {
            const int y = max(x + 1, yb * kPairBlock) + pl;
            if (y < min(ne, (yb + 1) * kPairBlock)) {
                const int i = V.occl[x], j = V.occl[y];
                const int row = i * n_so + j;
                b0 = T.row_off[row];
                len = T.row_off[row + 1] - b0;
                pk = (uint32_t)oslot[i] | ((uint32_t)oslot[j] << 16);
                sg = (uint32_t)(x * nb + yb);
            }
        }
        // rows with entries moved to the lowest lanes, in order (a forward
        // permute in which every lane takes part: the empty rows go above)
        const uint64_t nzm = __ballot(len > 0);
        const int nrows = __popcll(nzm);
        if (nrows == 0) continue;
        const int dst = (len > 0) ? (int)mask_below(nzm) : nrows + (int)mask_below(~nzm);
        b0 = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)b0);
        len = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)len);
        pk = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)pk);
        sg = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)sg);
        const uint32_t end = wave_scan_u32(len);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)end, nrows - 1);
        const uint32_t start = end - len;  // = tot in the lanes past the last row
        const uint32_t delta = b0 - start;  // table offset of stream position pos in the row: pos + delta
        for (uint32_t c = 0; c < tot && !found; c += kTileUnroll * kWave) {
            uint32_t off[kTileUnroll], pkv[kTileUnroll], sgv[kTileUnroll], abv[kTileUnroll];
#pragma unroll
            for (int u = 0; u < kTileUnroll; ++u) {
                const uint32_t cu = c + (uint32_t)(u * kWave), pos = cu + (uint32_t)l;
                off[u] = 0;  // entry 0 stands in for lanes without a candidate
                pkv[u] = 0;
                sgv[u] = 0;
                if (cu < tot) {
                    // the row of each lane's position: the row holding cu
                    // (the rows starting at or before it, less one) plus the
                    // rows starting in cu+1 .. pos, found from one marker
                    // byte per row start in this chunk; its data comes from
                    // the row's lane.  Bit 31 of pkv marks a candidate.
                    const int k0 = __popcll(__ballot(start <= cu)) - 1;
                    uint8_t* mk = mark + u * kWave;
                    const uint32_t rel = start - cu;
                    if (l < nrows && rel - 1u < (uint32_t)(kWave - 1)) mk[rel] = 1;
                    wave_lds_sync();
                    const uint64_t sm = __ballot(mk[l] != 0);
                    mk[l] = 0;
                    wave_lds_sync();
                    const int src = (k0 + (int)mask_below(sm >> 1)) << 2;
                    const uint32_t rdl = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)delta);
                    const uint32_t rpk = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)pk);
                    const uint32_t rsg = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)sg);
                    if (pos < tot) {
                        off[u] = pos + rdl;
                        pkv[u] = rpk | 0x80000000u;
                        sgv[u] = rsg;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kTileUnroll; ++u) abv[u] = T.dab[off[u]];
#pragma unroll
            for (int u = 0; u < kTileUnroll; ++u) {
                // both target orbitals empty: both their slots are -1, so the
                // sign bit of their AND, and with it the candidate bit, stays
                const uint32_t a = abv[u] & 0xFFFFu, b = abv[u] >> 16;
                const bool surv = ((int)(pkv[u] & (uint32_t)(oslot[a] & oslot[b])) < 0) && !found;
                const uint64_t m = __ballot(surv);
                if (surv) {
                    const uint32_t sq = (qh + qn + mask_below(m)) & (kQueue - 1);
                    q64[sq] = (uint64_t)off[u] | ((uint64_t)sgv[u] << 32);
                    qab[sq] = (uint64_t)abv[u] | ((uint64_t)(pkv[u] & 0x7FFFFFFFu) << 32);
                }
                qn += (uint32_t)__popcll(m);
                if (qn >= (uint32_t)kWave) {
                    if constexpr (DEFER) {
                        finish();
                        issue(kWave);
                    } else {
                        found = batch(kWave);
                    }
                    wave_lds_sync();  // the batch's queue reads precede later writes
                    qh = (qh + kWave) & (kQueue - 1);
                    qn -= kWave;
                }
            }
        }
        if (PICK) break;
    }
    if constexpr (DEFER) {
        finish();
        if (qn > 0) {
            issue((int)qn);
            finish();
        }
    } else if (!found && qn > 0) {
        found = batch((int)qn);
    }
    if (!PICK && cur_s >= 0) {
        const double tot = wave_total(acc);
        if (l == 0) segsum[cur_s] = tot;
    }
    wave_lds_sync();
    if (PICK && !found && last_l >= 0) {
        // rounding left the target past the segment's last running sum: take
        // its last candidate with a positive rate
        if (l == 0) {
            double term;
            int cp, cq, ca, cb;
            const double2 vk = *(const double2*)(T.dvK + 2 * (size_t)last_off);
            cand_eval<true, false, false, false, UHF>(T, V, last_off, 0u, last_ab, vk, term, cp, cq, ca, cb);
            pick[0] = 2; pick[1] = cp; pick[2] = cq; pick[3] = ca; pick[4] = cb;
        }
        found = true;
    }
    return found;
}

// In-place inclusive prefix sum of the first n entries of a wave's log.
__device__ __forceinline__ double log_prefix(double* a, int n) {
    const int l = lane_id();
    double carry = 0.0;
    for (int base = 0; base < n; base += kWave) {
        const int k = base + l;
        const double v = (k < n) ? a[k] : 0.0;
        const double x = wave_inclusive_scan(v) + carry;
        if (k < n) a[k] = x;
        carry = __shfl(x, kWave - 1, kWave);
    }
    wave_lds_sync();
    return carry;
}

enum { MODE_ELOC = 0, MODE_CTMC = 1, MODE_INIT = 2 };

// Occupancy target of the sweep kernel when the walker state lives in HBM,
// HW waves per SIMD, compiled for two values: 3 for systems without doubles
// (the Hubbard update stream is HBM-bound and runs faster with the registers
// of three waves), 4 for systems with doubles (their candidate gathers wait on
// L2 and MALL and gain from a fourth wave per SIMD, a few spills included).
// Walker state in LDS: four waves per SIMD (measured faster than the
// compiler's own choice of three up to 40 spin-orbitals, a few spills
// included); the 64-spin-orbital specialisation is left to the compiler (1).
constexpr int sweep_waves_target(int nso_t, bool small, int hw) {
    return small ? ((nso_t <= 40) ? 4 : 1) : hw;
}

// NSO_T, NE_T, NT_T: compile-time n_so, Ne and workgroup size of a size
// specialisation (0 = taken from the arguments at run time).  With them the
// LDS layout and loop bounds fold to constants.
// RT: element type of R (double: FP64 form; float: mixed form, where B, the
// update denominators and every accumulation stay FP64).
// sweep_body runs walker w of the walker set S (W walkers) on the calling
// workgroup.
template <int NSO_T, int NE_T, int NT_T, bool NW1, bool SMALL, typename RT, bool UHF = false, bool CPS = false>
__device__ __forceinline__ void sweep_body(const Tab& Targ, const Wk& S, int64_t W, int64_t w, int mode, int n_steps,
                                           uint64_t step0, uint64_t seed, int refresh_period, double* eloc_hist,
                                           double* t_hist, int64_t* pick_hist) {
    static_assert(!(UHF && SMALL), "spin-blocked orbitals keep the walker state in HBM");
    extern __shared__ __align__(16) unsigned char smem[];
    Tab T = Targ;
    // compiled without correlators: every correlator branch folds away (a
    // system with correlators runs the variants compiled with them)
    if constexpr (!CPS) T.ncorr = 0;
    if (NSO_T) {
        T.n_so = NSO_T;
        T.ne = NE_T;
        T.nw = (NSO_T + 63) / 64;
    }
    // wave index made explicitly wave-uniform so that everything derived from it
    // (stream ranges, group cursors, log bookkeeping) lives in scalar registers
    const int tid = threadIdx.x, nt = NT_T ? NT_T : (int)blockDim.x, l = tid & 63;
    const int wv = (int)__builtin_amdgcn_readfirstlane((uint32_t)(tid >> 6)), nwv = nt >> 6;
    const int n_so = T.n_so, ne = T.ne, nw = T.nw;
    // pairs of occupied slots; none when the table holds no doubles (Hubbard)
    const int gd = T.has_doubles ? ne * (ne - 1) / 2 : 0;
    T.G = ne + gd;
    const Lds L = lds_layout(n_so, ne, nw, nt, SMALL, (int)sizeof(RT), T.ncorr);
    constexpr bool MIXED = sizeof(RT) < sizeof(double);
    // mixed form with the state in HBM: R stored split (FP32 + bfloat16 remainder)
    constexpr bool SPLIT = MIXED && !SMALL;
    uint64_t* occw = (uint64_t*)(smem + L.occw);
    int* occl = (int*)(smem + L.occl);
    int* slot = (int*)(smem + L.slot);
    int* oslot = (int*)(smem + L.oslot);
    double* s = (double*)(smem + L.s);
    double* es = (double*)(smem + L.es);
    double* ies = (double*)(smem + L.ies);
    double* red = (double*)(smem + L.red);
    uint32_t* stmp = (uint32_t*)(smem + L.stmp);
    int* mi = (int*)(smem + L.mi);
    double* md = (double*)(smem + L.md);
    int* wst = (int*)(smem + L.wst);
    uint64_t* q64 = (uint64_t*)(smem + L.q64) + wv * kQueue;
    uint64_t* qab = (uint64_t*)(smem + L.qab) + wv * kQueue;
    uint8_t* mark = smem + L.mark + (size_t)wv * kTileUnroll * kWave;
    double* wtot = (double*)(smem + L.wtot);
    double* lsum = (double*)(smem + L.lsum);
    uint32_t* loff = (uint32_t*)(smem + L.loff);
    uint32_t* lg = (uint32_t*)(smem + L.lg);
    uint32_t* sgend = (uint32_t*)(smem + L.sgend);
    uint32_t* sdelta = (uint32_t*)(smem + L.sdelta);
    uint32_t* svend = (uint32_t*)(smem + L.svend);
    uint32_t* spq = (uint32_t*)(smem + L.spq);
    double* sfac = (double*)(smem + L.sfac);
    double* sies = (double*)(smem + L.sies);
    double* w1 = (double*)(smem + L.w1);
    double* w2 = (double*)(smem + L.w2);
    double* cRp = (double*)(smem + L.cRp);
    double* cRq = (double*)(smem + L.cRq);
    // theta[:, 0:Ne]: a copy in LDS for the small mixed form, else the table
    const bool th_lds = SMALL && MIXED;
    double* thl = (double*)(smem + L.thl);
    const double* th = th_lds ? thl : T.theta;
    const int ths = th_lds ? ne : n_so;
    double* cBp = (double*)(smem + L.cBp);
    double* cBq = (double*)(smem + L.cBq);
    int* ipiv = (int*)(smem + L.ipiv);
    uint32_t* dblk = (uint32_t*)(smem + L.dblk);
    double* fcol = (double*)(smem + L.fcol);
    uint32_t* cidx = (uint32_t*)(smem + L.cidx);
    double* cinv = (double*)(smem + L.cinv);
    RT *R, *Rh;
    uint16_t* Rlo = nullptr;
    double* B;
    double* Fk = nullptr;      // the walker's Fock-like singles elements (state in HBM, Coulomb-exchange vectors)
    uint64_t* ftag = nullptr;  // their tag: the occupation words they hold, the Hamiltonian's id, moves since built
    double* segsum = nullptr;  // rate sums of the doubles' pair segments (state in HBM)
    uint32_t *dgend = nullptr, *ddelta = nullptr, *dvend = nullptr, *dpq = nullptr;
    const int npb = pair_blocks(ne);
    if (SMALL) {
        R = (RT*)(smem + L.R);
        B = (double*)(smem + L.B);
        Rh = (RT*)(smem + L.Rh);
        dgend = (uint32_t*)(smem + L.dgend);
        ddelta = (uint32_t*)(smem + L.ddelta);
        dvend = (uint32_t*)(smem + L.dvend);
        dpq = (uint32_t*)(smem + L.dpq);
    } else {
        R = (RT*)S.R + (size_t)w * T.rrow * ne;
        if (SPLIT) Rlo = S.Rlo + (size_t)w * T.rrow * ne;
        B = S.B + (size_t)w * ne * ne;
        Rh = R;
        uint8_t* sc = S.scratch + (size_t)w * S.scratch_stride;
        if (T.has_sV && T.fock) {
            Fk = (double*)(sc + scratch_fock_offset(ne, nw));
            ftag = (uint64_t*)(sc + scratch_tag_offset(ne));
        }
        segsum = (double*)sc;
    }
    const StepView<RT> V{occl, es,   SMALL ? Rh : R, sgend, sdelta, svend, spq, sfac, dgend, ddelta, dvend, dpq, ies,
                         slot, cidx, cinv, Fk, sies};

    // ---------------------------------------------------------------- load
    if (th_lds)
        for (int k = tid; k < n_so * ne; k += nt) {
            const int a = k / ne, x = k - a * ne;
            thl[k] = T.theta[(size_t)a * n_so + x];
        }
    for (int k = tid; k < nw; k += nt) occw[k] = S.occ[(size_t)w * nw + k];
    if (tid == 0) mi[MI_ST] = (mode == MODE_INIT) ? 0 : (int)S.status[w];
    __syncthreads();
    if (mode == MODE_INIT) {
        // bits beyond n_so are ignored; a wrong electron count marks the walker
        if (tid == 0) {
            if ((n_so & 63) != 0) occw[nw - 1] &= (1ull << (n_so & 63)) - 1ull;
            int pop = 0, popa = 0;
            for (int k = 0; k < nw; ++k) {
                pop += __popcll(occw[k]);
                // alpha electrons: orbitals below n
                const int lo = 64 * k;
                if (lo < T.n) popa += __popcll(occw[k] & ((T.n - lo >= 64) ? ~0ull : ((1ull << (T.n - lo)) - 1ull)));
            }
            // spin-blocked orbitals also need na alpha electrons (slots [0, na)
            // alpha); a flagged walker is parked on a valid determinant
            const bool uhf = UHF;
            if (pop != ne || (uhf && popa != T.na)) {
                mi[MI_ST] = (int)VMC_ST_SINGULAR;
                for (int k = 0; k < nw; ++k) occw[k] = 0ull;
                for (int k = 0; k < ne; ++k) {
                    const int o = (uhf && k >= T.na) ? T.n + k - T.na : k;
                    occw[o >> 6] |= 1ull << (o & 63);
                }
            }
        }
        __syncthreads();
        for (int pp = tid; pp < n_so; pp += nt) {
            const bool occd = (occw[pp >> 6] >> (pp & 63)) & 1ull;
            int rank = 0;
            for (int k = 0; k < (pp >> 6); ++k) rank += __popcll(occw[k]);
            rank += __popcll(occw[pp >> 6] & ((1ull << (pp & 63)) - 1ull));
            oslot[pp] = occd ? rank : -1;
            if (occd && rank < ne) slot[rank] = pp;
        }
        __syncthreads();
        // refresh_period 0: the caller runs the separate refresh kernel next
        // (always, with spin-blocked orbitals)
        if (refresh_period > 0 && !UHF) refresh_state<RT, SPLIT>(T, slot, B, R, s, fcol, ipiv, mi, red, th, ths, Rlo);
    } else {
        for (int k = tid; k < ne; k += nt) slot[k] = S.slot_orb[(size_t)w * ne + k];
        for (int pp = tid; pp < n_so; pp += nt) {
            oslot[pp] = S.orb_slot[(size_t)w * n_so + pp];
            s[pp] = S.s[(size_t)w * n_so + pp];
        }
        if (SMALL) {
            const RT* Rg = (const RT*)S.R + (size_t)w * n_so * ne;
            const double* Bg = S.B + (size_t)w * ne * ne;
            for (int k = tid; k < n_so * ne; k += nt) R[k] = Rg[k];
            for (int k = tid; k < ne * ne; k += nt) B[k] = Bg[k];
        }
        __syncthreads();
    }
    // H_NN from scratch (at load and after every re-inversion); updated per move
    auto hnn_full = [&]() __attribute__((always_inline)) {
        double hp = 0.0;
        for (int x = tid; x < ne; x += nt) {
            const int i = slot[x];
            const double* Di = T.D + (size_t)i * n_so;
            hp += T.hdiag[i];
            for (int y = x + 1; y < ne; ++y) hp += Di[slot[y]];
        }
        const double h = block_total(hp, red);
        if (tid == 0) md[MD_HNN] = h;
        __syncthreads();
    };
    hnn_full();

    const int steps = (mode == MODE_CTMC) ? n_steps : 1;
    double el_last = 0.0, t_last = 0.0;
    int64_t code_last = 0;
    bool moved = false;     // block-uniform: some move changed the state
    bool fock_ok = false;   // block-uniform: Fk holds the elements of the current occupation
    uint64_t fock_moves = 0;  // thread 0: moves applied to Fk since it was built
    for (int k = 0; k < steps && mode != MODE_INIT; ++k) {
        const uint64_t gstep = step0 + (uint64_t)k;
        const bool singular = (mi[MI_ST] & (int)VMC_ST_SINGULAR) != 0;
        // ------------------------------------------------- per-step setup
        for (int pp = tid; pp < n_so; pp += nt) {
            es[pp] = exp(s[pp]);
            ies[pp] = exp(-s[pp]);
            if (!((occw[pp >> 6] >> (pp & 63)) & 1ull)) continue;
            int rank = 0;
            for (int q = 0; q < (pp >> 6); ++q) rank += __popcll(occw[q]);
            rank += __popcll(occw[pp >> 6] & ((1ull << (pp & 63)) - 1ull));
            occl[rank] = pp;
        }
        if (T.ncorr) cps_states(T, occw, cidx, cinv);
        __syncthreads();
        if (SMALL) {
            // Rh[p][a] = R[a][p] exp(s_a) exp(-s_i), i = slot[p]: the Jastrow
            // factors of the amplitude ratio folded into the rows and columns
            // of R (they factor out of every 1x1 and 2x2 minor)
            for (int idx = tid; idx < n_so * ne; idx += nt) {
                const int p = idx / n_so, a = idx - p * n_so;
                Rh[idx] = (RT)((double)R[idx] * es[a] * ies[slot[p]]);
            }
        }
        // group descriptors: row lengths padded to 64 (scanned into stream
        // ends), table bases (turned into offset deltas), valid ends, slots
        // and Jastrow factors
        for (int x = tid; x < ne; x += nt) {
            const int i = occl[x];
            const uint32_t b0 = T.s_off[i], len = T.s_off[i + 1] - b0;
            sdelta[x] = b0;
            svend[x] = len;
            sgend[x] = SMALL ? ((len + 63u) & ~63u) : len;  // unpadded in HBM layout (dense stream)
            spq[x] = (uint32_t)oslot[i];
            sfac[x] = ies[i];
            sies[x] = ies[slot[x]];
        }
        // doubles, state in LDS: blocks of 64 consecutive pairs, one per wave
        // at a time; pass 1 sums each block's padded lengths, the block sums
        // are scanned, pass 2 scans within the block and writes the
        // descriptors.  State in HBM: no descriptors (pair_tiles forms them
        // per segment); the segment rate sums start at zero.
        const int nblk = SMALL ? (gd + kWave - 1) / kWave : 0;
        if (!SMALL && gd > 0)
            for (int k2 = tid; k2 < ne * npb; k2 += nt) segsum[k2] = 0.0;
        auto pair_row = [&](int t, int& i, int& j, uint32_t& b0, uint32_t& len) __attribute__((always_inline)) {
            int x, y;
            pair_decode(t, ne, x, y);
            i = occl[x];
            j = occl[y];
            const int row = i * n_so + j;
            b0 = T.row_off[row];
            len = T.row_off[row + 1] - b0;
        };
        for (int bk = wv; bk < nblk; bk += nwv) {
            const int t = bk * kWave + l;
            uint32_t plen = 0;
            if (t < gd) {
                int i, j;
                uint32_t b0, len;
                pair_row(t, i, j, b0, len);
                plen = (len + 63u) & ~63u;
            }
            const uint32_t tot = wave_scan_u32(plen);
            if (l == kWave - 1) dblk[bk] = tot;
        }
        __syncthreads();
        if (wv == 0) {
            uint32_t carry = 0;
            for (int b0 = 0; b0 < nblk; b0 += kWave) {
                const int bk = b0 + l;
                const uint32_t v = (bk < nblk) ? dblk[bk] : 0u;
                const uint32_t incl = wave_scan_u32(v);
                if (bk < nblk) dblk[bk] = carry + incl - v;  // exclusive
                carry += (uint32_t)__shfl((int)incl, kWave - 1, kWave);
            }
            if (l == 0) dblk[nblk] = carry;
        }
        __syncthreads();
        for (int bk = wv; bk < nblk; bk += nwv) {
            const int t = bk * kWave + l;
            int i = 0, j = 0;
            uint32_t b0 = 0, len = 0, plen = 0;
            if (t < gd) {
                pair_row(t, i, j, b0, len);
                plen = (len + 63u) & ~63u;
            }
            const uint32_t end = dblk[bk] + wave_scan_u32(plen), start = end - plen;
            if (t < gd) {
                dgend[t] = end;
                ddelta[t] = b0 - start;
                dvend[t] = start + len;
                dpq[t] = (uint32_t)oslot[i] | ((uint32_t)oslot[j] << 16);
            }
        }
        __syncthreads();
        const uint32_t LS = uni(block_inclusive_scan(sgend, ne, stmp));
        const uint32_t LD = (gd > 0) ? uni(dblk[nblk]) : 0u;
        for (int x = tid; x < ne; x += nt) {
            const uint32_t ps = x ? sgend[x - 1] : 0u;
            sdelta[x] -= ps;
            svend[x] += ps;
        }
        __syncthreads();

        // Fock-like singles elements of the occupied rows: kept from the
        // previous launch when its tag names this occupation and Hamiltonian,
        // else built here; updated after every move below.  The tag is
        // cleared first and written back at the end only if the elements are
        // then current.
        if (Fk && k == 0) {
            if (tid == 0) {
                bool same = ftag[nw] == T.ham_id && ftag[nw + 1] < kFockRebuild;
                for (int q = 0; q < nw; ++q) same = same && ftag[q] == occw[q];
                mi[MI_FTAG] = same ? 1 : 0;
                fock_moves = same ? ftag[nw + 1] : 0ull;
                ftag[nw] = 0ull;
            }
            __syncthreads();
            if (!singular) {
                if (!mi[MI_FTAG]) fock_rows(T, Fk, occl, ne, occl, ne);
                fock_ok = true;
                __syncthreads();
            }
        }
        // ------------------------------------------------- local energy
        double el_lane = 0.0;
        if (!singular) {
            // contiguous, chunk-aligned ranges of each stream per wave (the
            // singles stream of the HBM layout ends anywhere in its last chunk)
            const uint32_t cs = (LS + 63u) >> 6, cd = LD >> 6;
            const uint32_t r0s = (uint32_t)(((uint64_t)cs * wv / nwv) << 6), r1s = (uint32_t)(((uint64_t)cs * (wv + 1) / nwv) << 6);
            const uint32_t r0d = (uint32_t)(((uint64_t)cd * wv / nwv) << 6), r1d = (uint32_t)(((uint64_t)cd * (wv + 1) / nwv) << 6);
            const int lb = wv * (kLogS + kLogD);
            int ns = 0, nd = 0;
            const uint64_t occ0 = occw[0];
            if (r0s < r1s) {
                const uint32_t g0 = find_group(sgend, (uint32_t)ne, r0s);
                stream_pass<false, false, NW1, SMALL, UHF>(T, V, occ0, occw, r0s, r1s, g0, (uint32_t)ne, r0s, q64, qab, el_lane, lsum + lb, loff + lb, lg + lb, kLogS, ns, 0.0, 0.0, false, nullptr);
            }
            if (SMALL && r0d < r1d) {
                const uint32_t g0 = find_group(dgend, (uint32_t)gd, r0d);
                stream_pass<true, false, NW1, SMALL, UHF>(T, V, occ0, occw, r0d, r1d, g0, (uint32_t)gd, r0d, q64, qab, el_lane, lsum + lb + kLogS, loff + lb + kLogS, lg + lb + kLogS, kLogD, nd, 0.0, 0.0, false, nullptr);
            }
            if (!SMALL && gd > 0)
                pair_tiles<false, UHF>(T, V, oslot, mark, q64, qab, el_lane, segsum, 0, 0, 0.0, 0.0, false, nullptr);
            // per-wave inclusive prefix sums of the two logs and their totals
            const double ts = log_prefix(lsum + lb, ns), td = log_prefix(lsum + lb + kLogS, nd);
            if (l == 0) {
                int* ws = wst + wv * 8;
                ws[WS_NS] = ns; ws[WS_R1S] = (int)r1s;
                ws[WS_ND] = nd; ws[WS_R1D] = (int)r1d;
                wtot[2 * wv] = ts;
                wtot[2 * wv + 1] = td;
            }
        } else if (l == 0) {
            int* ws = wst + wv * 8;
            ws[WS_NS] = 0; ws[WS_ND] = 0;
            wtot[2 * wv] = 0.0;
            wtot[2 * wv + 1] = 0.0;
        }
        const double el = singular ? NAN : (block_total(el_lane, red) + md[MD_HNN]);

        // ------------------------------------------ T and the pick location
        // T = sum of the per-wave log totals (singles then doubles, waves in
        // order); the target u*T is located first among those totals, then by
        // binary search in that wave's prefix-summed log.  Doubles with the
        // state in HBM: their part of T is the sum of the pair segments' rate
        // sums in canonical order (by x, the sums of row x of the segments
        // first), and u*T is located among the segments.
        const bool tiled = !SMALL && gd > 0;
        if (tiled && !singular) {
            for (int x = tid; x < ne; x += nt) {
                double rs = 0.0;
                for (int yb = 0; yb < npb; ++yb) rs += segsum[x * npb + yb];
                fcol[x] = rs;
            }
            __syncthreads();
        }
        if (tid == 0) {
            double Tt = 0.0;
            if (!singular) {
                for (int st = 0; st < 2; ++st)
                    for (int q = 0; q < nwv; ++q) Tt += wtot[2 * q + st];
                if (tiled)
                    for (int x = 0; x < ne; ++x) Tt += fcol[x];
            }
            md[MD_T] = Tt;
            mi[MI_PTYPE] = 0;
            mi[MI_FS] = -1;
            mi[MI_SDNOW] = 0;
            const bool okT0 = !singular && Tt > 0.0 && isfinite(Tt) && isfinite(el);
            if (!singular && !(isfinite(Tt) && isfinite(el))) mi[MI_ST] |= (int)VMC_ST_NONFINITE;
            else if (!singular && !(Tt > 0.0)) mi[MI_ST] |= (int)VMC_ST_EMPTY;
            if (okT0 && mode == MODE_CTMC) {
                const double target = ctmc_uniform(seed, (uint64_t)w, gstep) * Tt;
                md[MD_TARGET] = target;
                double run = 0.0, fbase = 0.0, lbase = 0.0;
                int fs = -1, fw = -1, ls_ = -1, lw_ = -1;
                for (int st = 0; st < 2 && fs < 0; ++st)
                    for (int q = 0; q < nwv && fs < 0; ++q) {
                        const double v = wtot[2 * q + st];
                        if (v > 0.0) { ls_ = st; lw_ = q; lbase = run; }
                        if (v > 0.0 && run + v > target) { fs = st; fw = q; fbase = run; }
                        else run += v;
                    }
                bool fb = false;
                if (tiled && fs < 0) {
                    // doubles: the row x of segments, then the segment, whose
                    // running sum first exceeds the target (or, after
                    // rounding, the last segment with a positive sum)
                    int fx = -1, lx = -1;
                    double xbase = 0.0;
                    for (int x = 0; x < ne && fx < 0; ++x) {
                        const double v = fcol[x];
                        if (v > 0.0) { lx = x; xbase = run; }
                        if (v > 0.0 && run + v > target) fx = x;
                        else run += v;
                    }
                    const bool xfb = fx < 0;
                    if (xfb) fx = lx;
                    if (fx >= 0) {
                        double sr = xfb ? xbase : run;
                        int fy = -1, ly = -1;
                        double ybase = sr;
                        for (int yb = 0; yb < npb && fy < 0; ++yb) {
                            const double v = segsum[fx * npb + yb];
                            if (v > 0.0) { ly = yb; ybase = sr; }
                            if (!xfb && v > 0.0 && sr + v > target) fy = yb;
                            else sr += v;
                        }
                        const bool yfb = fy < 0;
                        if (yfb) fy = ly;
                        mi[MI_FS] = 2;
                        mi[MI_FW] = fx;
                        mi[MI_FK] = fy;
                        mi[MI_FFB] = (xfb || yfb) ? 1 : 0;
                        md[MD_BASE] = yfb ? ybase : sr;
                    } else if (ls_ >= 0) {
                        fs = ls_; fw = lw_; fbase = lbase; fb = true;
                    }
                } else if (fs < 0 && ls_ >= 0) {
                    fs = ls_; fw = lw_; fbase = lbase; fb = true;
                }
                if (fs >= 0) {
                    const int n_ent = wst[fw * 8 + (fs ? WS_ND : WS_NS)];
                    const double* pre = lsum + fw * (kLogS + kLogD) + (fs ? kLogS : 0);
                    int fk;
                    if (!fb) {
                        // smallest e with fbase + pre[e] > target
                        int lo = 0, hi = n_ent - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (fbase + pre[mid] > target) hi = mid;
                            else lo = mid + 1;
                        }
                        fk = lo;
                    } else {
                        // last entry with a positive sum
                        fk = n_ent - 1;
                        while (fk > 0 && !(pre[fk] > pre[fk - 1])) --fk;
                    }
                    mi[MI_FS] = fs;
                    mi[MI_FW] = fw;
                    mi[MI_FK] = fk;
                    mi[MI_FFB] = fb ? 1 : 0;
                    md[MD_BASE] = fbase + (fk ? pre[fk - 1] : 0.0);
                }
            }
        }
        __syncthreads();
        const double Ttot = md[MD_T];
        const bool okT = !singular && Ttot > 0.0 && isfinite(Ttot) && isfinite(el);
        const double tres = okT ? 1.0 / Ttot : 0.0;
        el_last = el;
        t_last = tres;
        code_last = 0;
        if (mode == MODE_ELOC) break;

        // --------------------------------------------------------- pick
        if (okT && mi[MI_FS] >= 0) {
            if (wv == 0 && mi[MI_FS] == 2) {
                // doubles, state in HBM: re-walk the located pair segment
                const int fx = (int)uni((uint32_t)mi[MI_FW]), fy = (int)uni((uint32_t)mi[MI_FK]);
                const bool fb = uni((uint32_t)mi[MI_FFB]) != 0;
                double dummy = 0.0;
                pair_tiles<true, UHF>(T, V, oslot, mark, q64, qab, dummy, nullptr, fx, fy, md[MD_BASE], md[MD_TARGET],
                                      fb, mi + MI_PTYPE);
            } else if (wv == 0) {
                const int fs = (int)uni((uint32_t)mi[MI_FS]), fw = (int)uni((uint32_t)mi[MI_FW]);
                const int fk = (int)uni((uint32_t)mi[MI_FK]);
                const bool fb = uni((uint32_t)mi[MI_FFB]) != 0;
                const int b = fw * (kLogS + kLogD) + (fs ? kLogS : 0) + fk;
                const uint32_t o0 = loff[b], g0 = lg[b];
                const uint32_t p0 = o0 - (fs ? ddelta[g0] : sdelta[g0]);  // stream position of the entry's first candidate
                const uint32_t c0 = p0 & ~63u;
                const uint32_t r1 = (uint32_t)wst[fw * 8 + (fs ? WS_R1D : WS_R1S)];
                const double base = md[MD_BASE], target = md[MD_TARGET];
                double dummy = 0.0;
                int dn = 0;
                if (fs == 0)
                    stream_pass<false, true, NW1, SMALL, UHF>(T, V, occw[0], occw, c0, r1, g0, (uint32_t)ne, p0, q64, qab, dummy, nullptr, nullptr, nullptr, 0, dn, base, target, fb, mi + MI_PTYPE);
                else
                    stream_pass<true, true, NW1, SMALL, UHF>(T, V, occw[0], occw, c0, r1, g0, (uint32_t)gd, p0, q64, qab, dummy, nullptr, nullptr, nullptr, 0, dn, base, target, fb, mi + MI_PTYPE);
            }
            __syncthreads();
        }

        // -------------------------------------------------------- update
        const int ptype = mi[MI_PTYPE];
        if (ptype != 0) {
            const int p = mi[MI_PP], q = mi[MI_PQ], a = mi[MI_PA], b = mi[MI_PB];
            const int i = slot[p], j = (ptype == 2) ? slot[q] : -1;
            // rows a (and b) of R over the slots, w, in FP64: read from R (the
            // split storage of the mixed form with the state in HBM gives them
            // to about 2^-33), or in the small mixed form recomputed as
            // theta[a, 0:Ne] B from theta in LDS, one thread per slot
            const int rrow = UHF ? T.n : n_so;
            auto rval = [&](size_t idx) __attribute__((always_inline)) -> double {
                return SPLIT ? (double)R[idx] + (double)bf16_val(Rlo[idx]) : (double)R[idx];
            };
            for (int x = tid; x < ne; x += nt) {
                double ra, rb = 0.0;
                if (MIXED && SMALL) {
                    const double* tha = th + (size_t)a * ths;
                    const double* Bx = B + x * ne;
                    ra = 0.0;
                    for (int c = 0; c < ne; ++c) ra += tha[c] * Bx[c];
                    if (ptype == 2) {
                        const double* thb = th + (size_t)b * ths;
                        for (int c = 0; c < ne; ++c) rb += thb[c] * Bx[c];
                    }
                } else if (UHF) {
                    // spin-blocked: a slot of the other spin holds zero
                    const bool xb = x >= T.na;
                    ra = (xb == (a >= T.n)) ? rval(r_index_uhf(T, x, a)) : 0.0;
                    if (ptype == 2) rb = (xb == (b >= T.n)) ? rval(r_index_uhf(T, x, b)) : 0.0;
                } else {
                    ra = rval((size_t)x * n_so + a);
                    if (ptype == 2) rb = rval((size_t)x * n_so + b);
                }
                w1[x] = ra;
                w2[x] = rb;
            }
            for (int x = tid; x < ne; x += nt) {
                cBp[x] = B[p * ne + x];
                if (ptype == 2) cBq[x] = B[q * ne + x];
            }
            // old rows p (and q) of R over the orbitals (spin-blocked: over the
            // slot's own spin's n orbitals); not needed in the small mixed
            // form, where R is re-formed after the move
            if (!(MIXED && SMALL)) {
                for (int a2 = tid; a2 < rrow; a2 += nt) {
                    cRp[a2] = rval((size_t)p * rrow + a2);
                    if (ptype == 2) cRq[a2] = rval((size_t)q * rrow + a2);
                }
            }
            if (SPLIT) {
                // the Sherman-Morrison denominators in FP64 from B: entry (a', x)
                // of R is theta[a', 0:Ne] B[x, :] (spin-blocked: zero across the
                // spins, the dot over x's own block), one wave per entry
                __syncthreads();  // the rows above read w before it is overwritten
                const int nden = ptype == 2 ? 4 : 1;
                for (int e = wv; e < nden; e += nwv) {
                    const int ao = (e & 2) ? b : a, x = (e & 1) ? q : p;
                    const bool xb = UHF && x >= T.na;
                    double acc = 0.0;
                    if (!UHF || (xb == (ao >= T.n))) {
                        const int c0 = xb ? T.na : 0, c1 = (UHF && !xb) ? T.na : ne;
                        const double* ta = th + (size_t)ao * ths;
                        const double* Bx = B + x * ne;
                        for (int c = c0 + l; c < c1; c += kWave) acc += ta[c] * Bx[c];
                        acc = wave_total(acc);
                    }
                    if (l == 0) ((e & 2) ? w2 : w1)[x] = acc;
                }
            }
            // change of H_NN (sum over the unchanged occupied orbitals)
            double dh = 0.0;
            for (int x = tid; x < ne; x += nt) {
                if (x == p || (ptype == 2 && x == q)) continue;
                const int kk = slot[x];
                dh += T.D[(size_t)a * n_so + kk] - T.D[(size_t)i * n_so + kk];
                if (ptype == 2) dh += T.D[(size_t)b * n_so + kk] - T.D[(size_t)j * n_so + kk];
            }
            dh = block_total(dh, red);  // its barriers also publish the rows and copies above
            if (ptype == 1) {
                const double rho = w1[p];
                if (tid == 0 && fabs(rho) < T.small_den) {
                    mi[MI_ST] |= (int)VMC_ST_SMALLDEN;
                    mi[MI_SDNOW] = 1;
                }
                __syncthreads();
                for (int x = tid; x < ne; x += nt) w1[x] = (w1[x] - (x == p ? 1.0 : 0.0)) / rho;
                __syncthreads();
                // R[x][a'] -= R[a'][p] w_x;  B[x'][x] -= B[x][p] w_x'  (B column by slot)
                if (UHF) {
                    // one spin's block of R (its slots' rows) and of B
                    const int lo = (p >= T.na) ? T.na : 0, cnt = (p >= T.na) ? ne - T.na : T.na;
                    r_update<RT, false, SPLIT>(R + (size_t)lo * T.n, Rlo + (SPLIT ? (size_t)lo * T.n : 0), cnt, T.n,
                                               cRp, w1 + lo, nullptr, nullptr);
                    rank_update_ld<false>(B + (size_t)lo * ne + lo, cnt, cnt, ne, cBp + lo, w1 + lo, nullptr, nullptr);
                } else {
                    if (!(MIXED && SMALL)) r_update<RT, false, SPLIT>(R, Rlo, ne, n_so, cRp, w1, nullptr, nullptr);
                    rank_update<double, false>(B, ne, ne, cBp, w1, nullptr, nullptr);
                }
                if (tid == 0) md[MD_HNN] += dh + T.hdiag[a] - T.hdiag[i];
            } else {
                const double c00 = w1[p], c01 = w1[q], c10 = w2[p], c11 = w2[q];
                const double det = c00 * c11 - c10 * c01;
                if (tid == 0 && fabs(det) < T.small_den) {
                    mi[MI_ST] |= (int)VMC_ST_SMALLDEN;
                    mi[MI_SDNOW] = 1;
                }
                __syncthreads();
                for (int x = tid; x < ne; x += nt) {
                    const double ra = w1[x] - (x == p ? 1.0 : 0.0);
                    const double rb = w2[x] - (x == q ? 1.0 : 0.0);
                    w1[x] = (c11 * ra - c01 * rb) / det;
                    w2[x] = (-c10 * ra + c00 * rb) / det;
                }
                __syncthreads();
                if (UHF) {
                    const int na = T.na, nb = ne - T.na, n = T.n;
                    if ((p >= na) == (q >= na)) {
                        // same spin: rank 2 on that spin's blocks
                        const int lo = (p >= na) ? na : 0, cnt = (p >= na) ? nb : na;
                        r_update<RT, true, SPLIT>(R + (size_t)lo * n, Rlo + (SPLIT ? (size_t)lo * n : 0), cnt, n,
                                                  cRp, w1 + lo, cRq, w2 + lo);
                        rank_update_ld<true>(B + (size_t)lo * ne + lo, cnt, cnt, ne, cBp + lo, w1 + lo, cBq + lo,
                                             w2 + lo);
                    } else {
                        // opposite spins (p alpha, q beta): w1 vanishes on the
                        // beta slots and w2 on the alpha ones, so each spin's
                        // blocks take one rank-1 update
                        r_update<RT, false, SPLIT>(R, Rlo, na, n, cRp, w1, nullptr, nullptr);
                        r_update<RT, false, SPLIT>(R + (size_t)na * n, Rlo + (SPLIT ? (size_t)na * n : 0), nb, n,
                                                   cRq, w2 + na, nullptr, nullptr);
                        rank_update_ld<false>(B, na, na, ne, cBp, w1, nullptr, nullptr);
                        rank_update_ld<false>(B + (size_t)na * ne + na, nb, nb, ne, cBq + na, w2 + na, nullptr,
                                              nullptr);
                    }
                } else {
                    if (!(MIXED && SMALL)) r_update<RT, true, SPLIT>(R, Rlo, ne, n_so, cRp, w1, cRq, w2);
                    rank_update<double, true>(B, ne, ne, cBp, w1, cBq, w2);
                }
                if (tid == 0)
                    md[MD_HNN] += dh + T.hdiag[a] + T.hdiag[b] - T.hdiag[i] - T.hdiag[j] +
                                  T.D[(size_t)a * n_so + b] - T.D[(size_t)i * n_so + j];
            }
            if (MIXED && SMALL) {
                // small mixed form: FP32 R is not carried by the update at all;
                // it is re-formed from the FP64-exact B on the matrix cores,
                // one small GEMM per move from theta in LDS
                __syncthreads();
                r_gemm<RT>(T, B, R, th, ths);
            }
            // Jastrow sums s_p += J_pa [p!=a] - J_pi [p!=i] (+ the same for b, j)
            const double* Ja = T.J + (size_t)a * n_so;
            const double* Ji = T.J + (size_t)i * n_so;
            for (int pp = tid; pp < n_so; pp += nt) {
                double d = (pp != a ? Ja[pp] : 0.0) - (pp != i ? Ji[pp] : 0.0);
                if (ptype == 2) {
                    const double* Jb = T.J + (size_t)b * n_so;
                    const double* Jj = T.J + (size_t)j * n_so;
                    d += (pp != b ? Jb[pp] : 0.0) - (pp != j ? Jj[pp] : 0.0);
                }
                s[pp] += d;
            }
            __syncthreads();
            if (tid == 0) {
                occw[i >> 6] &= ~(1ull << (i & 63));
                occw[a >> 6] |= (1ull << (a & 63));
                oslot[i] = -1;
                oslot[a] = p;
                slot[p] = a;
                if (ptype == 2) {
                    occw[j >> 6] &= ~(1ull << (j & 63));
                    occw[b >> 6] |= (1ull << (b & 63));
                    oslot[j] = -1;
                    oslot[b] = q;
                    slot[q] = b;
                }
            }
            code_last = pack_pick(ptype, i, j, a, b);
            moved = true;
            __syncthreads();
            if (Fk) fock_move(T, Fk, slot, ne, i, ptype == 2 ? j : -1, a, ptype == 2 ? b : -1);
            ++fock_moves;
        }
        if (tid == 0) {
            if (eloc_hist) eloc_hist[(size_t)k * W + w] = el;
            if (t_hist) t_hist[(size_t)k * W + w] = tres;
            if (pick_hist) pick_hist[(size_t)k * W + w] = code_last;
        }
        // ------------------------------------------------------- refresh
        // periodic, or right after a move whose Sherman-Morrison denominator
        // was small (the update then amplified the rounding of B and R)
        if (refresh_period > 0 && !UHF && (((gstep + 1) % (uint64_t)refresh_period) == 0 || mi[MI_SDNOW])) {
            refresh_state<RT, SPLIT>(T, slot, B, R, s, fcol, ipiv, mi, red, th, ths, Rlo);
            hnn_full();
        }
    }

    // ---------------------------------------------------------- write back
    __syncthreads();
    if (mode != MODE_ELOC) {
        for (int k = tid; k < nw; k += nt) S.occ[(size_t)w * nw + k] = occw[k];
        for (int k = tid; k < ne; k += nt) S.slot_orb[(size_t)w * ne + k] = slot[k];
        for (int pp = tid; pp < n_so; pp += nt) {
            S.orb_slot[(size_t)w * n_so + pp] = oslot[pp];
            S.s[(size_t)w * n_so + pp] = s[pp];
        }
        if (SMALL) {
            RT* Rg = (RT*)S.R + (size_t)w * n_so * ne;
            double* Bg = S.B + (size_t)w * ne * ne;
            for (int k = tid; k < n_so * ne; k += nt) Rg[k] = R[k];
            for (int k = tid; k < ne * ne; k += nt) Bg[k] = B[k];
            // the split remainder starts at zero should the walkers later run
            // with their state in HBM (a batch)
            if (MIXED) {
                uint16_t* Lg = S.Rlo + (size_t)w * n_so * ne;
                for (int k = tid; k < n_so * ne; k += nt) Lg[k] = 0;
            }
        }
    }
    if (tid == 0) {
        if (fock_ok) {
            for (int q = 0; q < nw; ++q) ftag[q] = occw[q];
            ftag[nw] = T.ham_id;
            ftag[nw + 1] = fock_moves;
        }
        S.hnn[w] = md[MD_HNN];
        // walkers re-inverted by the separate refresh kernel carry updates
        // since their last inversion once they have moved
        if (mode == MODE_CTMC && !SMALL && refresh_period == 0 && moved) mi[MI_ST] |= (int)VMC_ST_STALE;
        S.status[w] = (uint32_t)mi[MI_ST];
        if (mode != MODE_INIT) {
            S.eloc[w] = el_last;
            S.tres[w] = t_last;
        }
        if (mode == MODE_CTMC) S.pick[w] = code_last;
        if (mode == MODE_INIT) S.pick[w] = 0;
    }
}

// One workgroup per walker of one system.
template <int NSO_T, int NE_T, int NT_T, bool NW1, bool SMALL, typename RT, bool UHF = false, int HW = 3,
          bool CPS = false>
__global__ void __launch_bounds__(NT_T ? NT_T : 512) __attribute__((amdgpu_waves_per_eu(sweep_waves_target(NSO_T, SMALL, HW))))
k_sweep(Tab T, Wk S, int64_t W, int mode, int n_steps, uint64_t step0, const uint64_t* step_dev, uint64_t seed,
        int refresh_period, double* eloc_hist, double* t_hist, int64_t* pick_hist) {
    const int64_t w = blockIdx.x;
    if (w >= W) return;
    // global step of the first move: step0, plus a device-resident counter
    // when the caller keeps one (graph replays advance it)
    const uint64_t s0 = step_dev ? step0 + *step_dev : step0;
    sweep_body<NSO_T, NE_T, NT_T, NW1, SMALL, RT, UHF, CPS>(T, S, W, w, mode, n_steps, s0, seed, refresh_period,
                                                       eloc_hist, t_hist, pick_hist);
}

__global__ void k_step_advance(uint64_t* step_dev, uint64_t n) {
    if (threadIdx.x == 0) *step_dev += n;
}

// Several systems of different sizes in one launch: workgroups [block0,
// block0 + W) of the grid belong to entry e.  Every system runs the variant
// with the walker state in HBM (any size, one layout per system, LDS sized
// for the largest) and refreshes in place; none carries correlators.
constexpr int kMaxBatch = 8;
struct BatchEntry {
    Tab T;
    Wk S;
    int64_t W, block0;
    uint64_t seed, step0;
    int refresh;
    double *eh, *th;
    int64_t* ph;
};
struct BatchArgs {
    BatchEntry e[kMaxBatch];
    int n;
};

template <typename RT, int HW>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(HW)))
k_sweep_batch(BatchArgs A, int mode, int n_steps) {
    const int64_t b = blockIdx.x;
    int e = 0;
    while (e + 1 < A.n && A.e[e + 1].block0 <= b) ++e;
    const int64_t w = b - A.e[e].block0;
    if (w >= A.e[e].W) return;
    const BatchEntry& E = A.e[e];
    sweep_body<0, 0, 0, false, false, RT>(E.T, E.S, E.W, w, mode, n_steps, E.step0, E.seed, E.refresh, E.eh, E.th,
                                          E.ph);
}

// Threads of the re-inversion kernel's workgroup (one walker each).
constexpr int kRefreshThreads = 512;

// Re-inversion with the matrix held in registers: Gauss-Jordan elimination
// with partial pivoting in exchange form (pivot rows are marked used, never
// swapped), on G = A^T, A = theta[occ, 0:Ne] (G[r][c] = theta[slot c][r]).
// Lane l holds rows l and l + 64, wave w the columns w, w + 8, ...: the owner
// wave of column k keeps it in register 0 (it rotates its registers by one
// after each column it owns), finds the pivot row p with a wave reduction,
// and publishes the column and 1/pivot in LDS; after one block barrier every
// wave reads the pivot row from its own lane p with readlane and updates its
// registers.  Step k exchanges x_k with y_{p_k}; after Ne steps
// M'[p_k][j] = G^-1[k][p_j].  The pivot row's own entry in the published
// column is pivot + 1, which turns the common update into the exchanged pivot
// row (v - (pv + 1) v / pv = -v / pv) with no per-lane case; G is scaled by a
// power of two to max |G| in [1/2, 1) so that the pivots, and the rounding of
// that form, stay of order one.
template <int RB>
__device__ __forceinline__ uint64_t pivot_key(double v, int r) {
    constexpr uint64_t m = (1ull << RB) - 1;
    const double a = fabs(v);
    const uint64_t bits = (a >= 0.0) ? (uint64_t)__double_as_longlong(a) : 0x7FF0000000000000ull;
    return (bits & ~m) | (uint64_t)((int)m - r);
}

__device__ __forceinline__ double readlane_d(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// LDS of the register Gauss-Jordan kernel: the inverse of an nm x nm matrix
// (theta[N], or the larger spin block) and slot lists of all Ne electrons.
__host__ __device__ inline size_t refresh_gj_lds_bytes(int nm, int ne) {
    const int cb = nm <= 128 ? 128 : 192;
    const size_t mat = nm <= 128 ? (size_t)nm * nm * 8 : 0, bufs = (size_t)(2 * cb + 4 + 2) * 8;
    return al16(mat > bufs ? mat : bufs) + 3 * al16((size_t)ne * 4) + al16((size_t)(kRefreshThreads / 64 + 2) * 8) +
           16;
}

// UHF (spin-blocked orbitals): one launch per spin (spin 0 alpha, 1 beta),
// each inverting that spin's diagonal block of theta[N] (slots and occupied
// columns [lo, lo + N_s)) and writing its rows of B (zero outside the block)
// and of R (own spin only); the beta launch, which runs second, also forms
// s and H_NN.  (Both spins in one launch of 2W workgroups measured slower.)
// General orbitals: one launch, spin unused.
template <typename RT, int H, int JC, bool UHF>
__global__ void __launch_bounds__(kRefreshThreads) __attribute__((amdgpu_waves_per_eu(H == 3 ? 2 : 4)))
k_refresh_gj(Tab T, Wk S, int64_t W, int spin, int lazy) {
    constexpr int NW = kRefreshThreads / 64;
    constexpr int CB = 64 * H;              // rows held by the lanes (one pivot-column buffer)
    constexpr int RB = H == 3 ? 8 : 7;      // bits of the row index in the pivot key
    static_assert(H * 64 <= 192 && NW * JC <= 192, "at most 192 rows and columns");
    static_assert(H < 3 || !UHF, "spin blocks of at most 128 electrons");
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t w = blockIdx.x;
    if (w >= W) return;
    // lazy: walkers that have not moved since their last inversion are
    // skipped (with spin-blocked orbitals the beta launch, which runs last,
    // clears the mark, so both launches see it)
    if (lazy && !(S.status[w] & VMC_ST_STALE)) return;
    const int ne_all = T.ne;
    const int lo = (UHF && spin) ? T.na : 0;
    const int tid = threadIdx.x, ne = UHF ? (spin ? ne_all - T.na : T.na) : ne_all, n_so = T.n_so, l = lane_id();
    const int wv = (int)uni((uint32_t)(tid >> 6));
    const int nm = UHF ? max(T.na, ne_all - T.na) : ne_all;  // the largest matrix of this system
    // B is staged in LDS for up to 128 rows; above that it goes straight to
    // the walker's buffer (160 x 160 FP64 would not fit)
    const size_t mat = (H == 3) ? 0 : (size_t)nm * nm * 8, bufs = (2 * CB + 4 + 2) * 8;
    size_t o = 0;
    double* Bs = (double*)smem;     // B (slot layout) once the elimination is done
    double* col = Bs;               // during it: the pivot column, two buffers
    double* pvb = Bs + 2 * CB;      // pivot and its reciprocal, two buffers
    int* pivb = (int*)(pvb + 4);    // pivot row, two buffers
    o += al16(mat > bufs ? mat : bufs);
    int* slot = (int*)(smem + o);
    o += al16((size_t)ne_all * 4);
    int* pk = (int*)(smem + o);  // pivot row of step k
    o += al16((size_t)ne_all * 4);
    int* qr = (int*)(smem + o);  // step at which row r was the pivot
    o += al16((size_t)ne_all * 4);
    double* red = (double*)(smem + o);
    o += al16((size_t)(kRefreshThreads / 64 + 2) * 8);
    int* flag = (int*)(smem + o);
    for (int k = tid; k < ne; k += kRefreshThreads) slot[k] = S.slot_orb[(size_t)w * ne_all + lo + k];
    if (tid == 0) flag[0] = (int)S.status[w];
    __syncthreads();
    double g[H][JC];
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < JC; ++j) {
        const int c = wv + NW * j;
        const double* tc = T.theta + (size_t)(c < ne ? slot[c] : 0) * n_so + lo;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int r = l + 64 * h;
            g[h][j] = (r < ne && c < ne) ? tc[r] : 0.0;
            mx = fmax(mx, fabs(g[h][j]));
        }
    }
    // scale by 2^-e with max |G| = m 2^e, m in [1/2, 1) (exact)
    mx = __longlong_as_double((long long)wave_max_u64((uint64_t)__double_as_longlong(mx)));
    if (l == 0) red[wv] = mx;
    __syncthreads();
    for (int q = 0; q < NW; ++q) mx = fmax(mx, red[q]);
    int ex = 0;
    if (mx > 0.0 && mx < INFINITY) frexp(mx, &ex);
    const double scale = ldexp(1.0, -ex);
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
        for (int j = 0; j < JC; ++j) g[h][j] *= scale;
    uint64_t used[H];  // rows already pivots, identical in every wave
#pragma unroll
    for (int h = 0; h < H; ++h) used[h] = 0;
    bool singular = false;
    int owned = 0;
    for (int k = 0; k < ne; ++k) {
        const int b = k & 1, ow = k % NW;
        if (wv == ow) {
            // pivot: the largest |G[r][k]| over unused rows as a u64 key (the
            // bits of |G[r][k]|, whose order is that of the values, with the
            // low RB mantissa bits replaced by 2^RB - 1 - r: values within
            // 2^(RB-52) of each other tie and the lowest r wins; a NaN counts
            // as the largest, so a poisoned matrix still pivots on an unused row)
            uint64_t key = 0;
#pragma unroll
            for (int h = 0; h < H; ++h)
                if (l + 64 * h < ne && !((used[h] >> l) & 1)) key = umax64(key, pivot_key<RB>(g[h][0], l + 64 * h));
            const int p = (int)((1u << RB) - 1) - (int)(wave_max_u64(key) & ((1u << RB) - 1));
            double pv = 0.0;
#pragma unroll
            for (int h = 0; h < H; ++h)
                if ((p >> 6) == h) pv = readlane_d(g[h][0], p & 63);
            const double ipv = (pv != 0.0) ? 1.0 / pv : 0.0;
            double* cw = col + b * CB;
#pragma unroll
            for (int h = 0; h < H; ++h) cw[l + 64 * h] = (l + 64 * h == p) ? pv + 1.0 : g[h][0];
            if (l == 0) {
                pvb[2 * b] = pv;
                pvb[2 * b + 1] = ipv;
                pivb[b] = p;
                pk[k] = p;
                qr[p] = k;
            }
        }
        __syncthreads();
        const int piv = (int)uni((uint32_t)pivb[b]);
        const double pv = pvb[2 * b], ipv = pvb[2 * b + 1];
#pragma unroll
        for (int h = 0; h < H; ++h)
            if ((piv >> 6) == h) used[h] |= 1ull << (piv & 63);
        singular |= !(fabs(pv) > 0.0) || !(fabs(pv) <= DBL_MAX);
        // every row: G[r][c] -= (G[r][k] / pv) G[p][c]; the pivot row reads
        // pv + 1 for G[p][k] and so becomes -G[p][c] / pv
        double t[H];
#pragma unroll
        for (int h = 0; h < H; ++h) t[h] = col[b * CB + l + 64 * h] * ipv;
        double v[JC];
        const int pl = piv & 63;
#pragma unroll
        for (int h = 0; h < H; ++h)
            if ((piv >> 6) == h) {
#pragma unroll
                for (int j = 0; j < JC; ++j) v[j] = readlane_d(g[h][j], pl);
            }
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
            for (int j = 0; j < JC; ++j) g[h][j] = fma(-t[h], v[j], g[h][j]);
        if (wv == ow) {  // column k becomes G[r][k] / pv, 1 / pv on the pivot row
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const double nk = (l + 64 * h == piv) ? ipv : t[h];
#pragma unroll
                for (int j = 0; j + 1 < JC; ++j) g[h][j] = g[h][j + 1];
                g[h][JC - 1] = nk;
            }
            ++owned;
        }
    }
    if (singular && tid == 0) flag[0] |= (int)VMC_ST_SINGULAR;
    __syncthreads();
    // B[p][x] = A^-1[x][p] = G^-1[p][x]: lane (r), register j (column c) holds
    // G^-1[q_r][p_c]; the registers have been rotated by the number of
    // columns this wave owned
    double* Bg = S.B + (size_t)w * ne_all * ne_all;
    double* Bo = (H == 3) ? Bg : Bs;  // general orbitals only when H == 3 (ne == ne_all)
#pragma unroll
    for (int j = 0; j < JC; ++j) {
        const int c = wv + NW * ((j + owned) % JC);
        if (c < ne) {
            const int pc = pk[c];
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int r = l + 64 * h;
                if (r < ne) Bo[(size_t)qr[r] * ne + pc] = g[h][j] * scale;
            }
        }
    }
    __syncthreads();
    RT* R = (RT*)S.R + (size_t)w * T.rrow * ne_all;
    constexpr bool SPLIT = sizeof(RT) < sizeof(double);
    uint16_t* Rlo = SPLIT ? S.Rlo + (size_t)w * T.rrow * ne_all : nullptr;
    if (!UHF) {
        if (H < 3)
            for (int k = tid; k < ne * ne; k += kRefreshThreads) Bg[k] = Bs[k];
        r_gemm_theta_regs<RT, 16 * H, SPLIT>(T, Bo, R, T.theta, n_so, Rlo);
    } else {
        // this spin's rows of B, zero outside the block
        for (int k = tid; k < ne * ne_all; k += kRefreshThreads) {
            const int p = k / ne_all, x = k - p * ne_all;
            Bg[(size_t)(lo + p) * ne_all + x] = (x >= lo && x < lo + ne) ? Bs[p * ne + x - lo] : 0.0;
        }
        // R rows of this spin's slots over its n orbitals: theta[own spin
        // rows][lo, lo + N_s) times the block inverse
        Tab Tb = T;
        Tb.ne = ne;
        Tb.n_so = T.n;
        r_gemm_theta_regs<RT, 16 * H, SPLIT>(Tb, Bs, R + (size_t)lo * T.n,
                                             T.theta + (size_t)(spin ? T.n : 0) * n_so + lo, n_so,
                                             SPLIT ? Rlo + (size_t)lo * T.n : nullptr);
        if (spin == 0) {
            if (tid == 0) S.status[w] = (uint32_t)flag[0];
            return;
        }
        // the beta launch: s and H_NN over every slot
        __syncthreads();
        for (int k = tid; k < ne_all; k += kRefreshThreads) slot[k] = S.slot_orb[(size_t)w * ne_all + k];
        __syncthreads();
    }
    double* sv = S.s + (size_t)w * n_so;
    for (int pp = tid; pp < n_so; pp += kRefreshThreads) {
        const double* Jr = T.J + (size_t)pp * n_so;
        double acc = 0.0;
        for (int k = 0; k < ne_all; ++k) {
            const int q = slot[k];
            if (q != pp) acc += Jr[q];
        }
        sv[pp] = acc;
    }
    double hp = 0.0;
    for (int x = tid; x < ne_all; x += kRefreshThreads) {
        const int i = slot[x];
        const double* Di = T.D + (size_t)i * n_so;
        hp += T.hdiag[i];
        for (int y = x + 1; y < ne_all; ++y) hp += Di[slot[y]];
    }
    const double hnn = block_total(hp, red);
    if (tid == 0) {
        S.hnn[w] = hnn;
        S.status[w] = (uint32_t)flag[0] & ~(uint32_t)VMC_ST_STALE;
    }
}

// Canonical candidate list of one walker (single wave, groups in order).
template <typename RT>
__global__ void __launch_bounds__(64) k_excitations(Tab T, Wk S, int64_t w, int32_t* ijab, double* hval, double* ratio,
                                                    int64_t cap, int64_t* count) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n_so = T.n_so, ne = T.ne, nw = T.nw, l = lane_id();
    uint64_t* occw = (uint64_t*)smem;
    int* occl = (int*)(smem + al16((size_t)nw * 8));
    int* oslot = occl + ((ne + 3) & ~3);
    double* es = (double*)(smem + al16((size_t)nw * 8) + al16((size_t)ne * 4) + al16((size_t)n_so * 4));
    double* ies = es + n_so;
    uint32_t* queue = (uint32_t*)(ies + n_so);
    double* cinv = (double*)(queue + kQueue);
    uint32_t* cidx = (uint32_t*)(cinv + T.ncorr);
    for (int k = l; k < nw; k += 64) occw[k] = S.occ[(size_t)w * nw + k];
    for (int pp = l; pp < n_so; pp += 64) {
        oslot[pp] = S.orb_slot[(size_t)w * n_so + pp];
        const double sv = S.s[(size_t)w * n_so + pp];
        es[pp] = exp(sv);
        ies[pp] = exp(-sv);
    }
    __syncthreads();
    for (int pp = l; pp < n_so; pp += 64)
        if (oslot[pp] >= 0) {
            int rank = 0;
            for (int q = 0; q < (pp >> 6); ++q) rank += __popcll(occw[q]);
            rank += __popcll(occw[pp >> 6] & ((1ull << (pp & 63)) - 1ull));
            occl[rank] = pp;
        }
    if (T.ncorr) cps_states(T, occw, cidx, cinv);
    __syncthreads();
    const RT* R = (const RT*)S.R + (size_t)w * T.rrow * ne;
    int64_t off = 0;
    for (int g = 0; g < T.G; ++g) {
        const Group Gr = group_of(T, g, occl, oslot, ies);
        auto ev = [&](uint32_t e, bool act) -> bool {
            if (act) {
                const int64_t pos = off + l;
                int a, b = -1;
                double r, h;
                if (Gr.type == 1) {
                    r = single_ratio(T, Gr, e, R, es, cidx, cinv, a);
                    h = single_h(T, Gr, e, occl);
                } else {
                    r = double_ratio(T, Gr, e, R, es, cidx, cinv, a, b);
                    h = T.dvK[2 * (size_t)(Gr.base + e)];
                }
                if (pos < cap) {
                    ijab[5 * pos + 0] = Gr.type;
                    ijab[5 * pos + 1] = Gr.i;
                    ijab[5 * pos + 2] = Gr.j;
                    ijab[5 * pos + 3] = a;
                    ijab[5 * pos + 4] = b;
                    hval[pos] = h;
                    ratio[pos] = r;
                }
            }
            off += __popcll(__ballot(act));
            return false;
        };
        if (Gr.type == 1) scan_group<false>(T, OccLds{occw}, Gr.base, Gr.len, queue, ev);
        else scan_group<true>(T, OccLds{occw}, Gr.base, Gr.len, queue, ev);
    }
    if (l == 0) count[0] = off;
}

// ------------------------------------------------------------ parameters
// Spin-blocked orbitals: theta[a][x] for the occupied columns x < Ne is kept
// where orbital a and column x have the same spin (columns [0, na) alpha,
// [na, Ne) beta) and set to zero elsewhere; one block per orbital row.
__global__ void k_theta_spin_blocks(double* th, int n, int na, int ne) {
    const int a = blockIdx.x, n_so = 2 * n;
    const bool ab = a >= n;
    for (int x = threadIdx.x; x < ne; x += blockDim.x)
        if ((x >= na) != ab) th[(size_t)a * n_so + x] = 0.0;
}

__global__ void k_dense_J(const double* Jp, double* J, int n_so) {
    const int p = blockIdx.x;
    const int64_t start = (int64_t)p * n_so - (int64_t)p * (p - 1) / 2;
    for (int q = p + threadIdx.x; q < n_so; q += blockDim.x) {
        const double v = Jp[start + (q - p)];
        J[(size_t)p * n_so + q] = v;
        J[(size_t)q * n_so + p] = v;
    }
}

// exp(J_aa + J_bb + J_ab - J_ii - J_jj + J_ij - J_ai - J_aj - J_bi - J_bj) per doubles entry
__global__ void k_doubles_K(const uint32_t* row_off, const uint32_t* dab, const double* J, double* dvK, int n_so) {
    const int row = blockIdx.x;
    const int i = row / n_so, j = row - i * n_so;
    if (j <= i) return;
    const uint32_t b0 = row_off[row], b1 = row_off[row + 1];
    const double* Ji = J + (size_t)i * n_so;
    const double* Jj = J + (size_t)j * n_so;
    for (uint32_t e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
        const uint32_t ab = dab[e];
        const int a = (int)(ab & 0xFFFFu), b = (int)(ab >> 16);
        const double* Ja = J + (size_t)a * n_so;
        const double* Jb = J + (size_t)b * n_so;
        const double kap = Ja[a] + Jb[b] + Ja[b] - Ji[i] - Jj[j] + Ji[j] - Ja[i] - Ja[j] - Jb[i] - Jb[j];
        dvK[2 * (size_t)e + 1] = exp(kap);
    }
}

// exp(J_aa - J_ii - J_ai) per singles entry
__global__ void k_singles_K(const uint32_t* s_off, const uint32_t* sa, const double* J, double* sK, int n_so) {
    const int i = blockIdx.x;
    const double* Ji = J + (size_t)i * n_so;
    for (uint32_t e = s_off[i] + threadIdx.x; e < s_off[i + 1]; e += blockDim.x) {
        const int a = (int)sa[e];
        sK[e] = exp(J[(size_t)a * n_so + a] - Ji[i] - Ji[a]);
    }
}

__global__ void k_uniforms(uint64_t seed, int64_t n, uint64_t step, double* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = ctmc_uniform(seed, (uint64_t)k, step);
}

// ------------------------------------------------------------ gradient ratios
__global__ void k_logderiv_dense(Tab T, Wk S, double* out, int64_t n_p) {
    const int64_t w = blockIdx.x;
    const int n_so = T.n_so, ne = T.ne, nw = T.nw;
    const uint64_t* occ = S.occ + (size_t)w * nw;
    double* o = out + (size_t)w * n_p;
    for (int p = threadIdx.x; p < n_so; p += blockDim.x) {
        const int64_t start = (int64_t)p * n_so - (int64_t)p * (p - 1) / 2;
        const bool np = (occ[p >> 6] >> (p & 63)) & 1ull;
        for (int q = p; q < n_so; ++q) {
            const bool nq = (occ[q >> 6] >> (q & 63)) & 1ull;
            o[start + (q - p)] = (np && nq) ? 1.0 : 0.0;
        }
    }
    const int64_t nj = (int64_t)n_so * (n_so + 1) / 2;
    const double* B = S.B + (size_t)w * ne * ne;
    const int32_t* oslot = S.orb_slot + (size_t)w * n_so;
    for (int64_t idx = threadIdx.x; idx < (int64_t)n_so * n_so; idx += blockDim.x) {
        const int k = (int)(idx / n_so), x = (int)(idx - (int64_t)k * n_so);
        const int sl = oslot[k];
        o[nj + idx] = (sl >= 0 && x < ne) ? B[(size_t)sl * ne + x] : 0.0;
    }
    if (T.ncorr) {
        // correlators: 1/c at the state each correlator sees, 0 elsewhere
        double* oc = o + nj + (int64_t)n_so * n_so;
        const int ncoef = T.coff[T.ncorr];
        for (int e = threadIdx.x; e < ncoef; e += blockDim.x) oc[e] = 0.0;
        __syncthreads();
        for (int lam = threadIdx.x; lam < T.ncorr; lam += blockDim.x) {
            int idx = 0, wt = 1;
            for (int m = 0; m < 5; ++m) {
                const int site = T.csite[5 * lam + m];
                if (site < 0) break;
                const int b = site + T.n;
                idx += wt * (int)(((occ[site >> 6] >> (site & 63)) & 1ull) + 2 * ((occ[b >> 6] >> (b & 63)) & 1ull));
                wt *= 4;
            }
            oc[T.coff[lam] + idx] = 1.0 / T.cc[T.coff[lam] + idx];
        }
    }
}

// Jastrow part of G = sum_w g_w O_w: G_J[p][q] = sum_w g_w n_p(w) n_q(w) for
// p <= q, i.e. Occ^T diag(g) Occ with Occ the W x n_so occupation matrix, a
// symmetric rank-W update on the FP64 matrix cores.  One workgroup per 16 x 16
// tile (pt <= qt) of G_J, four waves over contiguous walker ranges.  A wave
// loads 64 walkers at a time (lane = walker: the occupation words of the
// tile's rows and columns, and g_w) and feeds them to 16 mfma_f64_16x16x4
// steps, A[m][k] = g_w n_p and B[k][m] = n_q for walker k of the step; the
// four partial tiles are added in wave order, so the result is deterministic.
constexpr int kSyrkWaves = 4;
__global__ void __launch_bounds__(64 * kSyrkWaves) k_grad_J_syrk(Tab T, Wk S, int64_t W, const double* g,
                                                                 double* out, int accumulate) {
    __shared__ double part[kSyrkWaves][16][16];
    const int n_so = T.n_so, nw = T.nw, nt16 = (n_so + 15) >> 4;
    int t = blockIdx.x, pt = 0;
    while (t >= nt16 - pt) {
        t -= nt16 - pt;
        ++pt;
    }
    const int qt = pt + t;
    const int l = lane_id(), m = l & 15, kq = l >> 4;
    const int wv = (int)uni((uint32_t)(threadIdx.x >> 6));
    // a 16-aligned tile lies within one 64-bit occupation word
    const int wp = (pt * 16) >> 6, wq = (qt * 16) >> 6;
    const int bp = (pt * 16 + m) & 63, bq = (qt * 16 + m) & 63;
    const int64_t w0 = W * wv / kSyrkWaves, w1 = W * (wv + 1) / kSyrkWaves;
    Mma<double>::acc_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int64_t c = w0; c < w1; c += kWave) {
        const int64_t wl = c + l;
        uint64_t op = 0, oq = 0;
        double gv = 0.0;
        if (wl < w1) {
            op = S.occ[(size_t)wl * nw + wp];
            oq = S.occ[(size_t)wl * nw + wq];
            gv = g[wl];
        }
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const int src = 4 * st + kq;
            const uint64_t sp = ((uint64_t)(uint32_t)__shfl((int)(op >> 32), src, kWave) << 32) |
                                (uint32_t)__shfl((int)(uint32_t)op, src, kWave);
            const uint64_t sq = ((uint64_t)(uint32_t)__shfl((int)(oq >> 32), src, kWave) << 32) |
                                (uint32_t)__shfl((int)(uint32_t)oq, src, kWave);
            const double sg = __shfl(gv, src, kWave);
            const double a = ((sp >> bp) & 1ull) ? sg : 0.0;
            const double b = ((sq >> bq) & 1ull) ? 1.0 : 0.0;
            acc = Mma<double>::step(a, b, acc);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) part[wv][Mma<double>::row(kq, j)][m] = acc[j];
    __syncthreads();
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        const int r = e >> 4, cc = e & 15;
        const int p = pt * 16 + r, q = qt * 16 + cc;
        if (p >= n_so || q >= n_so || q < p) continue;
        double v = 0.0;
        for (int k = 0; k < kSyrkWaves; ++k) v += part[k][r][cc];
        double* o = out + (int64_t)p * n_so - (int64_t)p * (p - 1) / 2 + (q - p);
        *o = (accumulate ? *o : 0.0) + v;
    }
}

// Orbital part: G[k][x] = sum_w g_w B_w[slot_w(k)][x] over the walkers that
// hold orbital k (B column by slot: the row of slot s is contiguous over x),
// x < Ne; zero for x >= Ne.  One workgroup per orbital k, 16 waves over
// contiguous walker ranges, lanes over x (NR values each, Ne <= 64 NR).  A
// wave loads the slots and weights of 64 walkers at once (lane = walker),
// then accumulates the rows of those that hold k, several rows in flight
// (four, or fewer for long rows so that they stay in registers);
// walkers with g_w = 0 (flagged ones among them) are skipped, so a
// non-finite B of a flagged walker cannot reach G.  The 16 partial rows are
// added in wave order: deterministic.
constexpr int kGradWaves = 16;
template <int NR>
__global__ void __launch_bounds__(64 * kGradWaves) k_grad_theta_rows(Tab T, Wk S, int64_t W, const double* g,
                                                                     double* out, int64_t nj, int accumulate) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* buf = (double*)smem;  // Ne doubles
    const int k = blockIdx.x, n_so = T.n_so, ne = T.ne, l = lane_id();
    const int wv = (int)uni((uint32_t)(threadIdx.x >> 6));
    const int64_t w0 = W * wv / kGradWaves, w1 = W * (wv + 1) / kGradWaves;
    constexpr int UF = NR <= 4 ? 4 : NR <= 8 ? 2 : 1;  // rows in flight
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    for (int64_t c = w0; c < w1; c += kWave) {
        const int64_t wl = c + l;
        int sl = -1;
        double gv = 0.0;
        if (wl < w1) {
            sl = S.orb_slot[(size_t)wl * n_so + k];
            gv = g[wl];
        }
        uint64_t m = __ballot(sl >= 0 && gv != 0.0);
        while (m) {
            // up to UF walkers of this chunk at a time, their rows loaded together
            int jl[UF];
            int cnt = 0;
#pragma unroll
            for (int u = 0; u < UF; ++u) {
                jl[u] = 0;
                if (m) {
                    jl[u] = __ffsll((unsigned long long)m) - 1;
                    m &= m - 1;
                    ++cnt;
                }
            }
            double v[UF][NR];
            double gw[UF];
#pragma unroll
            for (int u = 0; u < UF; ++u) {
                gw[u] = 0.0;
                if (u < cnt) {
                    const int j = (int)uni((uint32_t)jl[u]);
                    const int slot = __builtin_amdgcn_readlane(sl, j);
                    gw[u] = readlane_d(gv, j);
                    const double* row = S.B + ((size_t)(c + j) * ne + slot) * ne;
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const int x = l + 64 * r;
                        v[u][r] = (x < ne) ? row[x] : 0.0;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < UF; ++u)
                if (u < cnt)
#pragma unroll
                    for (int r = 0; r < NR; ++r) acc[r] = fma(gw[u], v[u][r], acc[r]);
        }
    }
    for (int q = 0; q < kGradWaves; ++q) {
        if (wv == q)
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int x = l + 64 * r;
                if (x < ne) buf[x] = (q ? buf[x] : 0.0) + acc[r];
            }
        __syncthreads();
    }
    double* o = out + nj + (size_t)k * n_so;
    for (int x = threadIdx.x; x < n_so; x += blockDim.x) o[x] = (accumulate ? o[x] : 0.0) + ((x < ne) ? buf[x] : 0.0);
}

// Correlator part of G = sum_w g_w O_w: G[l][n] = (sum of g_w over the walkers
// whose correlator l is in state n) / c_l[n].  One workgroup per correlator,
// four waves over contiguous walker ranges; a wave reads the states and
// weights of 64 walkers at once (lane = walker) and adds them into its own LDS
// histogram in walker order (lane 0, one walker at a time); the four
// histograms are added in wave order.  Deterministic; walkers with g_w = 0
// add nothing.
constexpr int kCpsWaves = 4;
__global__ void __launch_bounds__(64 * kCpsWaves) k_grad_cps(Tab T, Wk S, int64_t W, const double* g, double* out,
                                                             int64_t off0, int accumulate) {
    __shared__ double hist[kCpsWaves][1024];
    const int lam = blockIdx.x, l = lane_id(), nw = T.nw;
    const int wv = (int)uni((uint32_t)(threadIdx.x >> 6));
    const int c0 = T.coff[lam], ns = T.coff[lam + 1] - c0;
    int st[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) st[m] = T.csite[5 * lam + m];
    for (int e = threadIdx.x; e < kCpsWaves * 1024; e += blockDim.x) (&hist[0][0])[e] = 0.0;
    __syncthreads();
    const int64_t w0 = W * wv / kCpsWaves, w1 = W * (wv + 1) / kCpsWaves;
    for (int64_t c = w0; c < w1; c += kWave) {
        const int64_t wl = c + l;
        int idx = 0;
        double gv = 0.0;
        if (wl < w1) {
            const uint64_t* occ = S.occ + (size_t)wl * nw;
            int wt = 1;
#pragma unroll
            for (int m = 0; m < 5; ++m)
                if (st[m] >= 0) {
                    const int a = st[m], b = st[m] + T.n;
                    idx += wt * (int)(((occ[a >> 6] >> (a & 63)) & 1ull) + 2 * ((occ[b >> 6] >> (b & 63)) & 1ull));
                    wt *= 4;
                }
            gv = g[wl];
        }
        const int cnt = (int)min<int64_t>(kWave, w1 - c);
        for (int j = 0; j < cnt; ++j) {
            const double gj = readlane_d(gv, j);
            const int ij = __builtin_amdgcn_readlane(idx, j);
            if (gj != 0.0 && l == 0) hist[wv][ij] += gj;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ns; e += blockDim.x) {
        double v = 0.0;
        for (int q = 0; q < kCpsWaves; ++q) v += hist[q][e];
        double* o = out + off0 + c0 + e;
        *o = (accumulate ? *o : 0.0) + v / T.cc[c0 + e];
    }
}

__global__ void k_amsgrad(int64_t n, double* p, double* m, double* v, double* vh, const double* g, double lr, double b1,
                          double b2, double delta, int literal) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double gk = g[k];
    const double mk = b1 * m[k] + (1.0 - b1) * gk;
    double vhk;
    if (literal) {
        vhk = fmax(vh[k], b2 * vh[k] + (1.0 - b2) * gk * gk);
    } else {
        const double vk = b2 * v[k] + (1.0 - b2) * gk * gk;
        v[k] = vk;
        vhk = fmax(vh[k], vk);
    }
    m[k] = mk;
    vh[k] = vhk;
    p[k] -= lr * mk / (sqrt(vhk) + delta);
}

// Residence-time weighted energy of the current states (one workgroup, fixed
// summation order): out = {sum t, sum t E_L, E = sum t E_L / sum t, walkers
// counted}; with g, the contraction weights of the covariance gradient
// g_w = 2 t_w (E_L,w - E) / sum t.  Walkers whose t is not positive or whose
// E_L is not finite (flagged states) carry no weight and get g_w = 0.
__global__ void __launch_bounds__(1024) k_estimate(const double* eloc, const double* tres, int64_t W, double* out,
                                                   double* g) {
    __shared__ double red[2][16];
    const int tid = threadIdx.x, nt = blockDim.x, l = tid & 63, wv = tid >> 6, nwv = nt >> 6;
    double st = 0.0, se = 0.0, sn = 0.0;
    for (int64_t k = tid; k < W; k += nt) {
        const double t = tres[k], e = eloc[k];
        if (t > 0.0 && isfinite(e)) {
            st += t;
            se += t * e;
            sn += 1.0;
        }
    }
    st = wave_total(st);
    se = wave_total(se);
    sn = wave_total(sn);
    __shared__ double rn[16];
    if (l == 0) {
        red[0][wv] = st;
        red[1][wv] = se;
        rn[wv] = sn;
    }
    __syncthreads();
    double T = 0.0, TE = 0.0, N = 0.0;
    for (int q = 0; q < nwv; ++q) {
        T += red[0][q];
        TE += red[1][q];
        N += rn[q];
    }
    const double E = (T > 0.0) ? TE / T : NAN;
    if (tid == 0) {
        out[0] = T;
        out[1] = TE;
        out[2] = E;
        out[3] = N;
    }
    if (g)
        for (int64_t k = tid; k < W; k += nt) {
            const double t = tres[k], e = eloc[k];
            g[k] = (t > 0.0 && isfinite(e) && T > 0.0) ? 2.0 * t * (e - E) / T : 0.0;
        }
}


// One snapshot of the covariance gradient over several sets of states: the
// weights t_w E_L,w and t_w of the current states (0 for flagged states, as in
// k_estimate), and the running sums acc = {sum t, sum t E_L, E, states}
// (reset: start them here), one workgroup in a fixed summation order.  With
// A = sum t E_L O and B = sum t O over all snapshots (the contracted backward
// with these two weights), G = 2 (A - E B) / sum t (k_gradient_combine).
__global__ void __launch_bounds__(1024) k_snapshot_weights(const double* eloc, const double* tres, int64_t W,
                                                           double* acc, double* g_te, double* g_t, int reset) {
    __shared__ double red[3][16];
    const int tid = threadIdx.x, nt = blockDim.x, l = tid & 63, wv = tid >> 6, nwv = nt >> 6;
    double st = 0.0, se = 0.0, sn = 0.0;
    for (int64_t k = tid; k < W; k += nt) {
        const double t = tres[k], e = eloc[k];
        const bool ok = t > 0.0 && isfinite(e);
        g_te[k] = ok ? t * e : 0.0;
        g_t[k] = ok ? t : 0.0;
        if (ok) {
            st += t;
            se += t * e;
            sn += 1.0;
        }
    }
    st = wave_total(st);
    se = wave_total(se);
    sn = wave_total(sn);
    if (l == 0) {
        red[0][wv] = st;
        red[1][wv] = se;
        red[2][wv] = sn;
    }
    __syncthreads();
    if (tid == 0) {
        double T = 0.0, TE = 0.0, N = 0.0;
        for (int q = 0; q < nwv; ++q) {
            T += red[0][q];
            TE += red[1][q];
            N += red[2][q];
        }
        if (!reset) {
            T += acc[0];
            TE += acc[1];
            N += acc[3];
        }
        acc[0] = T;
        acc[1] = TE;
        acc[2] = (T > 0.0) ? TE / T : NAN;
        acc[3] = N;
    }
}

// G_k = 2 (A_k - E B_k) / sum t with E = acc[2], sum t = acc[0] (0 when no
// state carried weight).
__global__ void k_gradient_combine(int64_t n, const double* a, const double* b, const double* acc, double* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double T = acc[0], E = acc[2];
    out[k] = (T > 0.0) ? 2.0 * (a[k] - E * b[k]) / T : 0.0;
}

}  // namespace

// =============================================================================
// Host side
// =============================================================================
struct vmc_ctx {
    int n = 0, n_so = 0, na = 0, nb = 0, ne = 0, nw = 0, G = 0, precision = 0, refresh = 50;
    bool uhf = false;  // spin-blocked orbitals (VMC_UHF)
    uint64_t seed = 0;
    double eps = 0.0;
    int device = 0;
    int block_threads = 0;  // 0 = automatic
    int64_t n_dent = 0, n_sent = 0;
    bool has_sV = true;
    bool fock = true;  // singles elements kept per walker (see Tab::fock)
    double small_den = 1e-8;  // see Tab::small_den
    uint64_t ham_id = 0;      // see Tab::ham_id
    int waves = 0;            // occupancy target of the HBM-layout sweep: 3, 4 waves per SIMD, or 0 (library's choice)
    uint32_t *d_row_off = nullptr, *d_dab = nullptr, *d_s_off = nullptr, *d_sa = nullptr;
    uint64_t* d_dmask = nullptr;
    double *d_dvK = nullptr, *d_sh = nullptr, *d_sV = nullptr, *d_sK = nullptr, *d_D = nullptr,
           *d_hdiag = nullptr, *d_J = nullptr, *d_theta = nullptr;
    bool params_set = false;
    // correlators (vmc_cps_init, vmc_set_cps)
    int ncorr = 0;
    int64_t n_coef = 0;
    int32_t *d_csite = nullptr, *d_coff = nullptr, *d_sc_off = nullptr;
    uint32_t* d_sc_list = nullptr;
    double* d_cc = nullptr;
    bool cps_set = false;
    std::string err;
};

struct vmc_host_tables {
    vmc::HostTables t;
};

struct vmc_batch_ctx {
    std::vector<vmc_ctx*> sys;
    int nt = 256;
    int precision = 0;
    int waves = 0;  // occupancy target of the sweep kernel (waves per SIMD): 3, 4, or 0 for the library's choice
    int mode = 0;   // VMC_BATCH_FUSED or VMC_BATCH_STREAMS
    // VMC_BATCH_STREAMS: one stream per system (default priority), forked from
    // and joined back to the caller's stream through events
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;
    hipEvent_t fork = nullptr;
};

namespace {
thread_local std::string g_err;

vmc_status fail(vmc_ctx* h, vmc_status st, const std::string& msg) {
    if (h) h->err = msg;
    g_err = msg;
    return st;
}

#define HIP_OR_FAIL(h, call)                                                                             \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return fail((h), VMC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

Tab make_tab(const vmc_ctx* h) {
    Tab T;
    T.n_so = h->n_so;
    T.ne = h->ne;
    T.nw = h->nw;
    T.G = h->G;
    T.n = h->n;
    T.na = h->na;
    T.uhf = h->uhf ? 1 : 0;
    T.rrow = h->uhf ? h->n : h->n_so;
    T.eps = h->eps;
    T.row_off = h->d_row_off;
    T.dab = h->d_dab;
    T.dmask = h->d_dmask;
    T.dvK = h->d_dvK;
    T.s_off = h->d_s_off;
    T.sa = h->d_sa;
    T.sh = h->d_sh;
    T.sV = h->d_sV;
    T.has_doubles = h->n_dent > 0 ? 1 : 0;
    T.has_sV = h->has_sV ? 1 : 0;
    T.fock = (h->has_sV && h->fock) ? 1 : 0;
    T.small_den = h->small_den;
    T.ham_id = h->ham_id;
    T.sK = h->d_sK;
    T.D = h->d_D;
    T.hdiag = h->d_hdiag;
    T.J = h->d_J;
    T.theta = h->d_theta;
    T.ncorr = h->ncorr;
    T.csite = h->d_csite;
    T.coff = h->d_coff;
    T.cc = h->d_cc;
    T.sc_off = h->d_sc_off;
    T.sc_list = h->d_sc_list;
    return T;
}

// the Fock-like elements are sized whatever the launch shape, so that a later
// vmc_set_launch cannot outgrow walkers allocated before it
int64_t scratch_bytes(const vmc_ctx* h) { return (int64_t)scratch_layout_bytes(h->ne, h->nw, h->has_sV ? h->n_sent : 0); }

// bytes per element of R: FP64 form 8, mixed form 4
size_t r_bytes(const vmc_ctx* h) { return h->precision == VMC_MIXED ? 4 : 8; }

vmc_status check_walkers(vmc_ctx* h, const vmc_walkers* w) {
    if (!w) return fail(h, VMC_E_ARG, "walkers is NULL");
    if (w->n_walkers <= 0 || w->n_walkers > (int64_t)INT_MAX) return fail(h, VMC_E_ARG, "n_walkers out of range");
    if (!w->occ_bits || !w->slot_orb || !w->orb_slot || !w->ainv || !w->r || !w->jsum || !w->hnn || !w->eloc ||
        !w->tres || !w->pick || !w->status || !w->scratch)
        return fail(h, VMC_E_ARG, "a walker field pointer is NULL");
    if (h->precision == VMC_MIXED && !w->rlo) return fail(h, VMC_E_ARG, "the mixed form needs the rlo field");
    if (!h->params_set) return fail(h, VMC_E_ARG, "vmc_set_params has not been called");
    if (h->ncorr > 0 && !h->cps_set) return fail(h, VMC_E_ARG, "vmc_set_cps has not been called");
    return VMC_OK;
}

Wk make_wk(const vmc_ctx* h, const vmc_walkers* w) {
    Wk S;
    S.occ = (uint64_t*)w->occ_bits;
    S.slot_orb = (int32_t*)w->slot_orb;
    S.orb_slot = (int32_t*)w->orb_slot;
    S.B = (double*)w->ainv;
    S.R = w->r;
    S.Rlo = (uint16_t*)w->rlo;
    S.s = (double*)w->jsum;
    S.hnn = (double*)w->hnn;
    S.eloc = (double*)w->eloc;
    S.tres = (double*)w->tres;
    S.pick = (int64_t*)w->pick;
    S.status = (uint32_t*)w->status;
    S.scratch = (uint8_t*)w->scratch;
    S.scratch_stride = scratch_bytes(h);
    return S;
}

// LDS per workgroup: the walker state is kept on chip when it fits 64 KB
// (several walkers per CU); otherwise the per-walker work arrays alone may use
// up to the 160 KB a gfx950 workgroup can address.
constexpr size_t kMaxLds = 64 * 1024;
constexpr size_t kMaxLdsHbm = 160 * 1024;

// Size specialisations of the sweep kernel: (n_so, Ne, threads).
struct SweepSpec {
    int n_so, ne, nt;
};
constexpr SweepSpec kSpecs[] = {{16, 8, 64}, {16, 8, 128}, {16, 8, 256}, {40, 20, 128}, {40, 20, 256}, {64, 32, 256}};

struct SweepArgs {
    int mode, n_steps, refresh;
    uint64_t step0;
    double *eh, *th;
    int64_t* ph;
    const uint64_t* step_dev;
};

template <int NSO, int NE, int NT, bool NW1, bool SM, typename RT, bool UHF = false, int HW = 3, bool CPS = false>
void launch_one(dim3 grid, dim3 block, size_t lds, hipStream_t st, const Tab& T, const Wk& S, const vmc_walkers* w,
                const SweepArgs& a, const vmc_ctx* h) {
    hipLaunchKernelGGL((k_sweep<NSO, NE, NT, NW1, SM, RT, UHF, HW, CPS>), grid, block, lds, st, T, S, w->n_walkers, a.mode,
                       a.n_steps, a.step0, a.step_dev, h->seed, a.refresh, a.eh, a.th, a.ph);
}

// Waves per SIMD of the HBM variant for this system: 4 with doubles, else 3.
// Occupancy target of the HBM-layout sweep (waves per SIMD, which fixes its
// register budget): the caller's or autotuner's choice, else 4 with doubles
// (the candidate gathers wait on the caches: more waves hide them, a few
// spills included) and 3 without (the Hubbard update stream keeps its
// registers).
int hbm_waves(const vmc_ctx* h) {
    if (h->ncorr > 0) return 3;  // the variants with correlators are compiled for 3 only
    return h->waves ? h->waves : (h->n_dent > 0 ? 4 : 3);
}
int batch_waves(const vmc_batch_ctx* b) {
    if (b->waves) return b->waves;
    for (const vmc_ctx* h : b->sys)
        if (h->n_dent > 0) return 4;
    return 3;
}

template <bool NW1, bool UHF, typename RT>
void launch_hbm(dim3 grid, dim3 block, size_t lds, hipStream_t st, const Tab& T, const Wk& S, const vmc_walkers* w,
                const SweepArgs& a, const vmc_ctx* h) {
    if (hbm_waves(h) == 4) launch_one<0, 0, 0, NW1, false, RT, UHF, 4>(grid, block, lds, st, T, S, w, a, h);
    else launch_one<0, 0, 0, NW1, false, RT, UHF, 3>(grid, block, lds, st, T, S, w, a, h);
}

template <typename RT>
void launch_prec(bool small, bool nw1, int nt, dim3 grid, dim3 block, size_t lds, hipStream_t st, const Tab& T,
                 const Wk& S, const vmc_walkers* w, const SweepArgs& a, const vmc_ctx* h) {
    auto spec = [&](int n_so, int ne, int c) { return small && h->n_so == n_so && h->ne == ne && nt == c; };
    // with correlators: the variants of any size compiled with them
    if (h->ncorr > 0) {
        if (small && nw1) launch_one<0, 0, 0, true, true, RT, false, 3, true>(grid, block, lds, st, T, S, w, a, h);
        else if (small) launch_one<0, 0, 0, false, true, RT, false, 3, true>(grid, block, lds, st, T, S, w, a, h);
        else if (h->uhf && nw1) launch_one<0, 0, 0, true, false, RT, true, 3, true>(grid, block, lds, st, T, S, w, a, h);
        else if (h->uhf) launch_one<0, 0, 0, false, false, RT, true, 3, true>(grid, block, lds, st, T, S, w, a, h);
        else if (nw1) launch_one<0, 0, 0, true, false, RT, false, 3, true>(grid, block, lds, st, T, S, w, a, h);
        else launch_one<0, 0, 0, false, false, RT, false, 3, true>(grid, block, lds, st, T, S, w, a, h);
        return;
    }
    // walker state in HBM (always, with spin-blocked orbitals)
    if (!small) {
        if (h->uhf && nw1) launch_hbm<true, true, RT>(grid, block, lds, st, T, S, w, a, h);
        else if (h->uhf) launch_hbm<false, true, RT>(grid, block, lds, st, T, S, w, a, h);
        else if (nw1) launch_hbm<true, false, RT>(grid, block, lds, st, T, S, w, a, h);
        else launch_hbm<false, false, RT>(grid, block, lds, st, T, S, w, a, h);
    } else if (spec(16, 8, 64)) launch_one<16, 8, 64, true, true, RT>(grid, block, lds, st, T, S, w, a, h);
    else if (spec(16, 8, 128)) launch_one<16, 8, 128, true, true, RT>(grid, block, lds, st, T, S, w, a, h);
    else if (spec(16, 8, 256)) launch_one<16, 8, 256, true, true, RT>(grid, block, lds, st, T, S, w, a, h);
    else if (spec(40, 20, 128)) launch_one<40, 20, 128, true, true, RT>(grid, block, lds, st, T, S, w, a, h);
    else if (spec(40, 20, 256)) launch_one<40, 20, 256, true, true, RT>(grid, block, lds, st, T, S, w, a, h);
    else if (spec(64, 32, 256)) launch_one<64, 32, 256, true, true, RT>(grid, block, lds, st, T, S, w, a, h);
    else if (nw1) launch_one<0, 0, 0, true, true, RT>(grid, block, lds, st, T, S, w, a, h);
    else launch_one<0, 0, 0, false, true, RT>(grid, block, lds, st, T, S, w, a, h);
}

// Geometry of the sweep launch for this system.
struct SweepGeom {
    int nt;
    bool small;
    size_t lds;
};
SweepGeom sweep_geom(const vmc_ctx* h) {
    SweepGeom g;
    g.nt = h->block_threads > 0 ? h->block_threads : 256;
    const int rb = (int)r_bytes(h);
    // spin-blocked orbitals: always the layout with the walker state in HBM
    g.small = !h->uhf && lds_layout(h->n_so, h->ne, h->nw, g.nt, true, rb, h->ncorr).total <= kMaxLds;
    g.lds = lds_layout(h->n_so, h->ne, h->nw, g.nt, g.small, rb, h->ncorr).total;
    return g;
}

// Walkers whose state lives in HBM are re-inverted by the separate register
// Gauss-Jordan kernel up to 192 electrons (128 per spin block); above that in
// place in the sweep.
constexpr size_t kMaxRefreshLds = 160 * 1024;
// Register Gauss-Jordan shape: 1 (Ne <= 64), 2 (Ne <= 128) or, for general
// orbitals, 3 (Ne <= 192) rows per lane; 0 where Ne is larger (re-inversion
// in place in the sweep, or B in LDS).
int refresh_gj_rows(int ne, bool uhf) { return ne <= 64 ? 1 : ne <= 128 ? 2 : (ne <= 192 && !uhf) ? 3 : 0; }

bool use_refresh_kernel(const vmc_ctx* h) {
    if (h->uhf) return true;  // always the register kernel, one spin block at a time
    return !sweep_geom(h).small && refresh_gj_rows(h->ne, false) != 0;
}


// Size of the matrices the register Gauss-Jordan kernel inverts: theta[N], or
// with spin-blocked orbitals the larger of its two spin blocks.
int gj_size(const vmc_ctx* h) { return h->uhf ? std::max(h->na, h->nb) : h->ne; }

// The register Gauss-Jordan kernel for a shape (rows 1 or 2), precision and
// orbital form.
const void* refresh_gj_kernel(int rows, bool mixed, bool uhf) {
    if (rows == 1) {
        if (mixed) return uhf ? (const void*)k_refresh_gj<float, 1, 8, true> : (const void*)k_refresh_gj<float, 1, 8, false>;
        return uhf ? (const void*)k_refresh_gj<double, 1, 8, true> : (const void*)k_refresh_gj<double, 1, 8, false>;
    }
    if (rows == 3) return mixed ? (const void*)k_refresh_gj<float, 3, 24, false> : (const void*)k_refresh_gj<double, 3, 24, false>;
    if (mixed) return uhf ? (const void*)k_refresh_gj<float, 2, 16, true> : (const void*)k_refresh_gj<float, 2, 16, false>;
    return uhf ? (const void*)k_refresh_gj<double, 2, 16, true> : (const void*)k_refresh_gj<double, 2, 16, false>;
}

vmc_status launch_refresh(vmc_ctx* h, vmc_walkers* w, hipStream_t st, bool lazy = false) {
    const int rows = refresh_gj_rows(gj_size(h), h->uhf);
    if (rows == 0) return fail(h, VMC_E_UNSUPPORTED, "no separate re-inversion kernel for this size");
    Tab Ta = make_tab(h);
    Wk Sa = make_wk(h, w);
    const dim3 grid((unsigned)w->n_walkers), block(kRefreshThreads);
    const bool mixed = h->precision == VMC_MIXED;
    const size_t b = refresh_gj_lds_bytes(gj_size(h), h->ne);
    int64_t Wa = w->n_walkers;
    // spin-blocked: the alpha block, then the beta block (stream order)
    int lz = lazy ? 1 : 0;
    for (int spin = 0; spin < (h->uhf ? 2 : 1); ++spin) {
        int sp = spin;
        void* args[] = {&Ta, &Sa, &Wa, &sp, &lz};
        HIP_OR_FAIL(h, hipLaunchKernel(refresh_gj_kernel(rows, mixed, h->uhf), grid, block, args, b, st));
    }
    return VMC_OK;
}

vmc_status launch_sweep(vmc_ctx* h, vmc_walkers* w, const SweepArgs& a, hipStream_t st) {
    const SweepGeom g = sweep_geom(h);
    if (g.lds > kMaxLdsHbm) return fail(h, VMC_E_UNSUPPORTED, "system too large for the per-walker LDS budget");
    const bool nw1 = (h->nw == 1);
    const Tab T = make_tab(h);
    const Wk S = make_wk(h, w);
    const dim3 grid((unsigned)w->n_walkers), block((unsigned)g.nt);
    if (h->precision == VMC_MIXED)
        launch_prec<float>(g.small, nw1, g.nt, grid, block, g.lds, st, T, S, w, a, h);
    else
        launch_prec<double>(g.small, nw1, g.nt, grid, block, g.lds, st, T, S, w, a, h);
    HIP_OR_FAIL(h, hipGetLastError());
    return VMC_OK;
}

template <class T>
vmc_status upload(vmc_ctx* h, T** dst, const std::vector<T>& src, hipStream_t st) {
    const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    if (hipMalloc((void**)dst, bytes) != hipSuccess) return fail(h, VMC_E_OOM, "hipMalloc failed for a table");
    if (!src.empty()) HIP_OR_FAIL(h, hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return VMC_OK;
}

void free_ctx(vmc_ctx* h) {
    if (!h) return;
    void* ptrs[] = {h->d_row_off, h->d_dab,   h->d_dmask, h->d_s_off, h->d_sa,   h->d_dvK,    h->d_sh,
                    h->d_sV,      h->d_sK,    h->d_D,     h->d_hdiag, h->d_J,    h->d_theta,  h->d_csite,
                    h->d_coff,    h->d_sc_off, h->d_sc_list, h->d_cc};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete h;
}

vmc_status validate_desc(const vmc_system_desc* d) {
    if (!d) return fail(nullptr, VMC_E_ARG, "desc is NULL");
    if (d->n_orb <= 0 || 2 * d->n_orb > 1024) return fail(nullptr, VMC_E_ARG, "n_orb must be in 1..512");
    if (d->n_alpha < 0 || d->n_beta < 0 || d->n_alpha > d->n_orb || d->n_beta > d->n_orb ||
        d->n_alpha + d->n_beta < 1)
        return fail(nullptr, VMC_E_ARG, "electron counts out of range");
    if (d->n_alpha + d->n_beta > 2 * d->n_orb - 1)
        return fail(nullptr, VMC_E_ARG, "at least one empty spin-orbital is required");
    if (d->precision != VMC_FP64 && d->precision != VMC_MIXED)
        return fail(nullptr, VMC_E_ARG, "precision must be VMC_FP64 or VMC_MIXED");
    if (d->refresh_period < 1) return fail(nullptr, VMC_E_ARG, "refresh_period must be >= 1");
    if (d->orbitals != VMC_GHF && d->orbitals != VMC_UHF)
        return fail(nullptr, VMC_E_ARG, "orbitals must be VMC_GHF or VMC_UHF");
    return VMC_OK;
}

// Workspace of vmc_ctmc_step_static: the kernels' per-walker scratch (pair
// descriptors, singles elements) for callers that cannot allocate.  Each GPU
// holds its own copy of the array, at its own address, from module load until
// the process ends.  In host code the array's name is only a stand-in: its
// device address on each device comes from hipGetSymbolAddress, taken once
// per device by vmc_init with that device current, and only that address is
// ever passed to a kernel.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Address of this device's copy of the static workspace (set-up, once per
// device; the caller has made `device` current).
vmc_status static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(nullptr, VMC_E_UNSUPPORTED, "device index beyond 64");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return VMC_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(nullptr, VMC_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return VMC_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* vmc_last_error(vmc_handle h) { return h ? h->err.c_str() : g_err.c_str(); }

void vmc_decode_pick(int64_t code, int32_t out5[5]) {
    if (!out5) return;
    const int type = (int)(code >> 48);
    out5[0] = type;
    if (type == 0) {
        out5[1] = out5[2] = out5[3] = out5[4] = -1;
        return;
    }
    out5[1] = (int)((code >> 36) & 0xFFF);
    out5[2] = (type == 2) ? (int)((code >> 24) & 0xFFF) : -1;
    out5[3] = (int)((code >> 12) & 0xFFF);
    out5[4] = (type == 2) ? (int)(code & 0xFFF) : -1;
}

vmc_status vmc_host_tables_build(const vmc_system_desc* desc, const double* h1, const vmc_eri_list* eri, double eps,
                                 vmc_host_tables** out) {
    if (!out) return fail(nullptr, VMC_E_ARG, "out is NULL");
    *out = nullptr;
    vmc_status st = validate_desc(desc);
    if (st != VMC_OK) return st;
    if (!eri) return fail(nullptr, VMC_E_ARG, "eri list is NULL");
    vmc_host_tables* t = new vmc_host_tables;
    const std::string e =
        build_host_tables(desc->n_orb, desc->n_alpha, desc->n_beta, h1, eri->n_nz, eri->pqrs, eri->val, eps, t->t);
    if (!e.empty()) {
        delete t;
        return fail(nullptr, VMC_E_ARG, e);
    }
    *out = t;
    return VMC_OK;
}

vmc_status vmc_host_tables_sizes(const vmc_host_tables* t, int64_t out[2]) {
    if (!t || !out) return fail(nullptr, VMC_E_ARG, "NULL argument");
    out[0] = (int64_t)t->t.dv.size();
    out[1] = (int64_t)t->t.sa.size();
    return VMC_OK;
}

vmc_status vmc_host_tables_get(const vmc_host_tables* t, int64_t* row_off, int32_t* dab, double* dv, int64_t* s_off,
                               int32_t* sa, double* sS, double* sh) {
    if (!t) return fail(nullptr, VMC_E_ARG, "tables is NULL");
    const auto& T = t->t;
    if (row_off) std::memcpy(row_off, T.row_off.data(), T.row_off.size() * sizeof(int64_t));
    if (dab) std::memcpy(dab, T.dab.data(), T.dab.size() * sizeof(int32_t));
    if (dv) std::memcpy(dv, T.dv.data(), T.dv.size() * sizeof(double));
    if (s_off) std::memcpy(s_off, T.s_off.data(), T.s_off.size() * sizeof(int64_t));
    if (sa) std::memcpy(sa, T.sa.data(), T.sa.size() * sizeof(int32_t));
    if (sS) std::memcpy(sS, T.sS.data(), T.sS.size() * sizeof(double));
    if (sh) std::memcpy(sh, T.sh.data(), T.sh.size() * sizeof(double));
    return VMC_OK;
}

void vmc_host_tables_free(vmc_host_tables* t) { delete t; }

// Id of a new system's Hamiltonian (never 0): a random 32-bit prefix drawn
// once per process, then a counter, so no two systems of the process share
// one, and a walker scratch left by another process almost surely matches none.
static uint64_t next_ham_id() {
    static std::mutex mu;
    static uint64_t prefix = 0, count = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (prefix == 0) {
        std::random_device rd;
        prefix = (uint64_t)(rd() | 1u) << 32;
    }
    return prefix | (++count & 0xFFFFFFFFull);
}

vmc_status vmc_init(const vmc_system_desc* desc, const double* h1, const vmc_eri_list* eri, double eps,
                    hipStream_t stream, vmc_handle* out) {
    if (!out) return fail(nullptr, VMC_E_ARG, "out is NULL");
    *out = nullptr;
    vmc_status st = validate_desc(desc);
    if (st != VMC_OK) return st;
    if (!eri) return fail(nullptr, VMC_E_ARG, "eri list is NULL");
    vmc::HostTables T;
    const std::string e =
        build_host_tables(desc->n_orb, desc->n_alpha, desc->n_beta, h1, eri->n_nz, eri->pqrs, eri->val, eps, T);
    if (!e.empty()) return fail(nullptr, VMC_E_ARG, e);
    if (T.dv.size() >= (size_t)UINT32_MAX || T.sa.size() >= (size_t)UINT32_MAX)
        return fail(nullptr, VMC_E_UNSUPPORTED, "table larger than 2^32 entries");
    if (desc->orbitals == VMC_UHF) {
        // the spin-blocked layout keeps one spin per slot: every kept
        // excitation must move each electron within its own spin
        if (refresh_gj_rows(std::max(desc->n_alpha, desc->n_beta), true) == 0)
            return fail(nullptr, VMC_E_UNSUPPORTED, "VMC_UHF supports at most 128 electrons of each spin");
        const int n = desc->n_orb, n_so = 2 * n;
        auto beta = [n](int o) { return o >= n; };
        for (int i = 0; i < n_so; ++i)
            for (int64_t k = T.s_off[i]; k < T.s_off[i + 1]; ++k)
                if (beta((int)T.sa[k]) != beta(i))
                    return fail(nullptr, VMC_E_ARG, "VMC_UHF needs spin-conserving singles");
        for (int i = 0; i < n_so; ++i)
            for (int j = i + 1; j < n_so; ++j)
                for (int64_t k = T.row_off[(size_t)i * n_so + j]; k < T.row_off[(size_t)i * n_so + j + 1]; ++k)
                    if (beta((int)T.dab[2 * k]) != beta(i) || beta((int)T.dab[2 * k + 1]) != beta(j))
                        return fail(nullptr, VMC_E_ARG, "VMC_UHF needs spin-conserving doubles");
    }
    vmc_ctx* h = new vmc_ctx;
    h->ham_id = next_ham_id();
    h->n = desc->n_orb;
    h->n_so = 2 * h->n;
    h->na = desc->n_alpha;
    h->nb = desc->n_beta;
    h->ne = h->na + h->nb;
    h->nw = (h->n_so + 63) / 64;
    h->G = h->ne + h->ne * (h->ne - 1) / 2;
    h->precision = desc->precision;
    h->uhf = desc->orbitals == VMC_UHF;
    h->refresh = desc->refresh_period;
    h->seed = desc->seed;
    h->eps = eps;
    h->n_dent = (int64_t)T.dv.size();
    h->n_sent = (int64_t)T.sa.size();
    h->has_sV = false;
    for (double v : T.sV)
        if (v != 0.0) {
            h->has_sV = true;
            break;
        }
    if (hipGetDevice(&h->device) != hipSuccess) {
        free_ctx(h);
        return fail(nullptr, VMC_E_HIP, "hipGetDevice failed");
    }
    {
        const vmc_status ss = static_scratch_setup(h->device);
        if (ss != VMC_OK) {
            const std::string msg = g_err;
            free_ctx(h);
            return fail(nullptr, ss, msg);
        }
    }
    std::vector<uint32_t> row_off(T.row_off.begin(), T.row_off.end());
    std::vector<uint32_t> dab(T.dv.size());
    for (size_t k = 0; k < T.dv.size(); ++k) dab[k] = (uint32_t)T.dab[2 * k] | ((uint32_t)T.dab[2 * k + 1] << 16);
    std::vector<uint32_t> s_off(T.s_off.begin(), T.s_off.end());
    std::vector<uint32_t> sa(T.sa.begin(), T.sa.end());
    std::vector<double> dvK(2 * T.dv.size(), 0.0), zeross(T.sa.size(), 0.0);
    for (size_t k = 0; k < T.dv.size(); ++k) dvK[2 * k] = T.dv[k];
    // occupancy masks of the doubles targets, for systems that fit one 64-bit word
    std::vector<uint64_t> dmask;
    if (h->n_so <= 64) {
        dmask.resize(T.dv.size());
        for (size_t k = 0; k < T.dv.size(); ++k)
            dmask[k] = (1ull << T.dab[2 * k]) | (1ull << T.dab[2 * k + 1]);
    }
    vmc_status u = VMC_OK;
    if ((u = upload(h, &h->d_row_off, row_off, stream)) != VMC_OK ||
        (u = upload(h, &h->d_dab, dab, stream)) != VMC_OK ||
        (h->n_so <= 64 && (u = upload(h, &h->d_dmask, dmask, stream)) != VMC_OK) || (u = upload(h, &h->d_dvK, dvK, stream)) != VMC_OK || (u = upload(h, &h->d_s_off, s_off, stream)) != VMC_OK ||
        (u = upload(h, &h->d_sa, sa, stream)) != VMC_OK || (u = upload(h, &h->d_sh, T.sh, stream)) != VMC_OK ||
        (u = upload(h, &h->d_sV, T.sV, stream)) != VMC_OK || (u = upload(h, &h->d_sK, zeross, stream)) != VMC_OK ||
        (u = upload(h, &h->d_D, T.D, stream)) != VMC_OK || (u = upload(h, &h->d_hdiag, T.hdiag, stream)) != VMC_OK) {
        std::string msg = h->err;
        free_ctx(h);
        return fail(nullptr, u, msg);
    }
    if (hipMalloc((void**)&h->d_J, sizeof(double) * h->n_so * h->n_so) != hipSuccess ||
        hipMalloc((void**)&h->d_theta, sizeof(double) * h->n_so * h->n_so) != hipSuccess) {
        free_ctx(h);
        return fail(nullptr, VMC_E_OOM, "hipMalloc failed for parameters");
    }
    if (hipStreamSynchronize(stream) != hipSuccess) {
        free_ctx(h);
        return fail(nullptr, VMC_E_HIP, "table upload failed");
    }
    // dynamic LDS beyond 64 KB for the kernels that may need it, set here once
    // so that later calls (possibly under graph capture) only launch
    {
        const void* big[] = {(const void*)k_sweep<0, 0, 0, false, false, double, false, 3>,
                             (const void*)k_sweep<0, 0, 0, true, false, double, false, 3>,
                             (const void*)k_sweep<0, 0, 0, false, false, float, false, 3>,
                             (const void*)k_sweep<0, 0, 0, true, false, float, false, 3>,
                             (const void*)k_sweep<0, 0, 0, false, false, double, true, 3>,
                             (const void*)k_sweep<0, 0, 0, true, false, double, true, 3>,
                             (const void*)k_sweep<0, 0, 0, false, false, float, true, 3>,
                             (const void*)k_sweep<0, 0, 0, true, false, float, true, 3>,
                             (const void*)k_sweep<0, 0, 0, false, false, double, false, 4>,
                             (const void*)k_sweep<0, 0, 0, true, false, double, false, 4>,
                             (const void*)k_sweep<0, 0, 0, false, false, float, false, 4>,
                             (const void*)k_sweep<0, 0, 0, true, false, float, false, 4>,
                             (const void*)k_sweep<0, 0, 0, false, false, double, true, 4>,
                             (const void*)k_sweep<0, 0, 0, true, false, double, true, 4>,
                             (const void*)k_sweep<0, 0, 0, false, false, float, true, 4>,
                             (const void*)k_sweep<0, 0, 0, true, false, float, true, 4>,
                             (const void*)k_sweep<0, 0, 0, false, false, double, false, 3, true>,
                             (const void*)k_sweep<0, 0, 0, true, false, double, false, 3, true>,
                             (const void*)k_sweep<0, 0, 0, false, false, float, false, 3, true>,
                             (const void*)k_sweep<0, 0, 0, true, false, float, false, 3, true>,
                             (const void*)k_sweep<0, 0, 0, false, false, double, true, 3, true>,
                             (const void*)k_sweep<0, 0, 0, true, false, double, true, 3, true>,
                             (const void*)k_sweep<0, 0, 0, false, false, float, true, 3, true>,
                             (const void*)k_sweep<0, 0, 0, true, false, float, true, 3, true>,
                             (const void*)k_sweep_batch<double, 4>, (const void*)k_sweep_batch<float, 4>,
                             (const void*)k_sweep_batch<double, 3>, (const void*)k_sweep_batch<float, 3>};
        for (const void* f : big) {
            const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLdsHbm);
            if (e != hipSuccess) {
                free_ctx(h);
                return fail(nullptr, VMC_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
            }
        }
    }
    {
        hipError_t e = hipSuccess;
        const bool mixed = h->precision == VMC_MIXED;
        const size_t gj = refresh_gj_lds_bytes(gj_size(h), h->ne);
        if (e == hipSuccess && refresh_gj_rows(gj_size(h), h->uhf) != 0 && gj <= kMaxRefreshLds)
            e = hipFuncSetAttribute(refresh_gj_kernel(refresh_gj_rows(gj_size(h), h->uhf), mixed, h->uhf),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)gj);
        if (e != hipSuccess) {
            free_ctx(h);
            return fail(nullptr, VMC_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
        }
    }
    *out = h;
    return VMC_OK;
}

vmc_status vmc_set_params(vmc_handle h, const double* J_dev, const double* theta_dev, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    if (!J_dev || !theta_dev) return fail(h, VMC_E_ARG, "parameter pointer is NULL");
    const int n_so = h->n_so;
    HIP_OR_FAIL(h, hipMemcpyAsync(h->d_theta, theta_dev, sizeof(double) * n_so * n_so, hipMemcpyDeviceToDevice, st));
    if (h->uhf) {
        hipLaunchKernelGGL(k_theta_spin_blocks, dim3(n_so), dim3(64), 0, st, h->d_theta, h->n, h->na, h->ne);
        HIP_OR_FAIL(h, hipGetLastError());
    }
    hipLaunchKernelGGL(k_dense_J, dim3(n_so), dim3(256), 0, st, J_dev, h->d_J, n_so);
    HIP_OR_FAIL(h, hipGetLastError());
    if (h->n_dent > 0) {
        hipLaunchKernelGGL(k_doubles_K, dim3(n_so * n_so), dim3(64), 0, st, h->d_row_off, h->d_dab, h->d_J, h->d_dvK,
                           n_so);
        HIP_OR_FAIL(h, hipGetLastError());
    }
    if (h->n_sent > 0) {
        hipLaunchKernelGGL(k_singles_K, dim3(n_so), dim3(64), 0, st, h->d_s_off, h->d_sa, h->d_J, h->d_sK, n_so);
        HIP_OR_FAIL(h, hipGetLastError());
    }
    h->params_set = true;
    return VMC_OK;
}

vmc_status vmc_cps_init(vmc_handle h, int32_t n_corr, const int32_t* sites) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    if (h->ncorr > 0) return fail(h, VMC_E_ARG, "correlators are already set for this handle");
    if (n_corr < 1 || n_corr >= (1 << 24) || !sites) return fail(h, VMC_E_ARG, "n_corr must be in 1..2^24-1 with sites");
    const int n = h->n;
    std::vector<int32_t> csite((size_t)5 * n_corr), coff((size_t)n_corr + 1, 0), sc_off((size_t)n + 1, 0);
    std::vector<std::vector<uint32_t>> per_site((size_t)n);
    int64_t total = 0;
    for (int l = 0; l < n_corr; ++l) {
        int k = 0;
        while (k < 5 && sites[5 * l + k] >= 0) ++k;
        if (k == 0) return fail(h, VMC_E_ARG, "correlator " + std::to_string(l) + " has no site");
        for (int m = 0; m < 5; ++m) {
            const int st = (m < k) ? sites[5 * l + m] : -1;
            if (m < k && st >= n) return fail(h, VMC_E_ARG, "correlator " + std::to_string(l) + ": site out of range");
            for (int m2 = 0; m2 < m && m < k; ++m2)
                if (csite[5 * l + m2] == st) return fail(h, VMC_E_ARG, "correlator " + std::to_string(l) + ": repeated site");
            csite[5 * (size_t)l + m] = st;
            if (m < k) per_site[st].push_back((uint32_t)l | ((uint32_t)m << 24));
        }
        total += (int64_t)1 << (2 * k);
        if (total >= INT_MAX) return fail(h, VMC_E_UNSUPPORTED, "too many correlator coefficients");
        coff[l + 1] = (int32_t)total;
    }
    std::vector<uint32_t> sc_list;
    for (int st = 0; st < n; ++st) {
        sc_off[st] = (int32_t)sc_list.size();
        sc_list.insert(sc_list.end(), per_site[st].begin(), per_site[st].end());
    }
    sc_off[n] = (int32_t)sc_list.size();
    vmc_status u = VMC_OK;
    if ((u = upload(h, &h->d_csite, csite, nullptr)) != VMC_OK || (u = upload(h, &h->d_coff, coff, nullptr)) != VMC_OK ||
        (u = upload(h, &h->d_sc_off, sc_off, nullptr)) != VMC_OK ||
        (u = upload(h, &h->d_sc_list, sc_list, nullptr)) != VMC_OK)
        return u;
    if (hipMalloc((void**)&h->d_cc, sizeof(double) * (size_t)total) != hipSuccess)
        return fail(h, VMC_E_OOM, "hipMalloc failed for correlator coefficients");
    HIP_OR_FAIL(h, hipStreamSynchronize(nullptr));
    h->ncorr = n_corr;
    h->n_coef = total;
    h->cps_set = false;
    return VMC_OK;
}

vmc_status vmc_set_cps(vmc_handle h, const double* coeffs_dev, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    if (h->ncorr == 0) return fail(h, VMC_E_ARG, "vmc_cps_init has not been called");
    if (!coeffs_dev) return fail(h, VMC_E_ARG, "coefficient pointer is NULL");
    HIP_OR_FAIL(h, hipMemcpyAsync(h->d_cc, coeffs_dev, sizeof(double) * (size_t)h->n_coef, hipMemcpyDeviceToDevice, st));
    h->cps_set = true;
    return VMC_OK;
}

vmc_status vmc_cps_info(vmc_handle h, int64_t out[2]) {
    if (!h || !out) return fail(h, VMC_E_ARG, "NULL argument");
    out[0] = h->ncorr;
    out[1] = h->n_coef;
    return VMC_OK;
}

vmc_status vmc_walker_bytes(vmc_handle h, int64_t W, size_t fb[VMC_NFIELDS]) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    if (!fb || W <= 0) return fail(h, VMC_E_ARG, "bad arguments");
    const size_t w = (size_t)W;
    fb[VMC_F_OCC] = w * h->nw * 8;
    fb[VMC_F_SLOT_ORB] = w * h->ne * 4;
    fb[VMC_F_ORB_SLOT] = w * h->n_so * 4;
    fb[VMC_F_AINV] = w * h->ne * h->ne * 8;
    fb[VMC_F_R] = w * h->ne * (h->uhf ? h->n : h->n_so) * r_bytes(h);
    fb[VMC_F_RLO] = h->precision == VMC_MIXED ? w * h->ne * (h->uhf ? h->n : h->n_so) * 2 : 0;
    fb[VMC_F_JSUM] = w * h->n_so * 8;
    fb[VMC_F_HNN] = w * 8;
    fb[VMC_F_ELOC] = w * 8;
    fb[VMC_F_TRES] = w * 8;
    fb[VMC_F_PICK] = w * 8;
    fb[VMC_F_STATUS] = w * 4;
    fb[VMC_F_SCRATCH] = w * (size_t)scratch_bytes(h);
    return VMC_OK;
}

vmc_status vmc_walkers_init(vmc_handle h, vmc_walkers* w, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    vmc_status s = check_walkers(h, w);
    if (s != VMC_OK) return s;
    w->since_inv = 0;
    if (use_refresh_kernel(h)) {
        s = launch_sweep(h, w, SweepArgs{MODE_INIT, 1, 0, w->step, nullptr, nullptr, nullptr, nullptr}, st);
        return s != VMC_OK ? s : launch_refresh(h, w, st);
    }
    return launch_sweep(h, w, SweepArgs{MODE_INIT, 1, h->refresh, w->step, nullptr, nullptr, nullptr, nullptr}, st);
}

vmc_status vmc_walkers_refresh(vmc_handle h, vmc_walkers* w, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    vmc_status s = check_walkers(h, w);
    if (s != VMC_OK) return s;
    // HBM-resident walkers: the refresh kernel, slots kept; otherwise a fresh
    // initialisation
    w->since_inv = 0;
    if (use_refresh_kernel(h)) return launch_refresh(h, w, st);
    return launch_sweep(h, w, SweepArgs{MODE_INIT, 1, h->refresh, w->step, nullptr, nullptr, nullptr, nullptr}, st);
}

vmc_status vmc_local_energy(vmc_handle h, vmc_walkers* w, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    vmc_status s = check_walkers(h, w);
    if (s != VMC_OK) return s;
    return launch_sweep(h, w, SweepArgs{MODE_ELOC, 1, h->refresh, w->step, nullptr, nullptr, nullptr, nullptr}, st);
}

vmc_status vmc_ctmc_step(vmc_handle h, vmc_walkers* w, int32_t n_steps, double* eh, double* th, int64_t* ph,
                         hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    vmc_status s = check_walkers(h, w);
    if (s != VMC_OK) return s;
    if (n_steps < 0) return fail(h, VMC_E_ARG, "n_steps must be >= 0");
    if (n_steps == 0) return VMC_OK;
    if (!use_refresh_kernel(h)) {
        s = launch_sweep(h, w, SweepArgs{MODE_CTMC, n_steps, h->refresh, w->step, eh, th, ph, nullptr}, st);
        if (s == VMC_OK) w->step += (uint64_t)n_steps;
        return s;
    }
    // segments of at most refresh_period moves since the last inversion; the
    // refresh kernel runs before a move that would exceed that
    const int64_t W = w->n_walkers;
    const uint64_t S = (uint64_t)h->refresh;
    int k = 0;
    while (k < n_steps) {
        if (w->since_inv >= S) {
            if ((s = launch_refresh(h, w, st)) != VMC_OK) return s;
            w->since_inv = 0;
        }
        const uint64_t g = w->step;
        const int seg = (int)std::min<uint64_t>((uint64_t)(n_steps - k), S - w->since_inv);
        s = launch_sweep(h, w, SweepArgs{MODE_CTMC, seg, 0, g, eh ? eh + (size_t)k * W : nullptr,
                                         th ? th + (size_t)k * W : nullptr, ph ? ph + (size_t)k * W : nullptr,
                                         nullptr}, st);
        if (s != VMC_OK) return s;
        w->step += (uint64_t)seg;
        w->since_inv += (uint64_t)seg;
        k += seg;
    }
    return VMC_OK;
}

vmc_status vmc_ctmc_step_static(vmc_handle h, vmc_walkers* w, int32_t n_steps, double* eh, double* th, int64_t* ph,
                                hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    if (!w) return fail(h, VMC_E_ARG, "walkers is NULL");
    if (w->n_walkers <= 0 || w->n_walkers > (int64_t)INT_MAX) return fail(h, VMC_E_ARG, "n_walkers out of range");
    const size_t need = (size_t)w->n_walkers * (size_t)scratch_bytes(h);
    if (need > kStaticScratchBytes)
        return fail(h, VMC_E_ARG, "the static workspace holds " + std::to_string(kStaticScratchBytes) + " bytes; " +
                                      std::to_string(w->n_walkers) + " walkers of this system need " +
                                      std::to_string(need));
    int dev = -1;
    HIP_OR_FAIL(h, hipGetDevice(&dev));
    if (dev != h->device) return fail(h, VMC_E_ARG, "the handle belongs to another device than the current one");
    void* ptr = (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
    if (!ptr) return fail(h, VMC_E_STATE, "static workspace not set up on this device");
    // the same sweep with the workspace field pointing at this device's copy
    // of the static array (every kernel rewrites what it reads of it first:
    // nothing needs clearing)
    vmc_walkers ws = *w;
    ws.scratch = ptr;
    const vmc_status s = vmc_ctmc_step(h, &ws, n_steps, eh, th, ph, st);
    w->step = ws.step;
    w->since_inv = ws.since_inv;
    return s;
}

vmc_status vmc_ctmc_step_dev(vmc_handle h, vmc_walkers* w, int32_t n_steps, uint64_t* step_dev, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    vmc_status s = check_walkers(h, w);
    if (s != VMC_OK) return s;
    if (!step_dev) return fail(h, VMC_E_ARG, "step_dev is NULL");
    if (n_steps < 0) return fail(h, VMC_E_ARG, "n_steps must be >= 0");
    if (n_steps == 0) return VMC_OK;
    if (!use_refresh_kernel(h)) {
        s = launch_sweep(h, w, SweepArgs{MODE_CTMC, n_steps, h->refresh, 0, nullptr, nullptr, nullptr, step_dev}, st);
    } else {
        if (n_steps % h->refresh != 0)
            return fail(h, VMC_E_ARG, "with the separate refresh kernel, n_steps must be a multiple of refresh_period");
        // before every segment of refresh_period moves, a lazy re-inversion:
        // walkers marked STALE (moved since their last inversion) are
        // re-inverted, fresh ones skip it, whatever state a replay finds
        for (int k = 0; k < n_steps && s == VMC_OK; k += h->refresh) {
            s = launch_refresh(h, w, st, true);
            if (s == VMC_OK)
                s = launch_sweep(h, w, SweepArgs{MODE_CTMC, h->refresh, 0, (uint64_t)k, nullptr, nullptr, nullptr,
                                                 step_dev}, st);
        }
        w->since_inv = (uint64_t)h->refresh;
    }
    if (s != VMC_OK) return s;
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, st, step_dev, (uint64_t)n_steps);
    HIP_OR_FAIL(h, hipGetLastError());
    return VMC_OK;
}

vmc_status vmc_excitations(vmc_handle h, const vmc_walkers* w, int64_t walker, int32_t* ijab, double* hval,
                           double* ratio, int64_t cap, int64_t* count, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    vmc_status s = check_walkers(h, w);
    if (s != VMC_OK) return s;
    if (walker < 0 || walker >= w->n_walkers) return fail(h, VMC_E_ARG, "walker index out of range");
    if (!count || cap < 0 || (cap > 0 && (!ijab || !hval || !ratio))) return fail(h, VMC_E_ARG, "bad output buffers");
    const size_t lds = al16((size_t)h->nw * 8) + al16((size_t)h->ne * 4) + al16((size_t)h->n_so * 4) +
                       2 * (size_t)h->n_so * 8 + (size_t)kQueue * 4 + (size_t)h->ncorr * 12;
    if (h->precision == VMC_MIXED)
        hipLaunchKernelGGL(k_excitations<float>, dim3(1), dim3(64), lds, st, make_tab(h), make_wk(h, w), walker, ijab,
                           hval, ratio, cap, count);
    else
        hipLaunchKernelGGL(k_excitations<double>, dim3(1), dim3(64), lds, st, make_tab(h), make_wk(h, w), walker, ijab,
                           hval, ratio, cap, count);
    HIP_OR_FAIL(h, hipGetLastError());
    return VMC_OK;
}

vmc_status vmc_uniforms(uint64_t seed, int64_t n, uint64_t step, double* out, hipStream_t st) {
    if (n <= 0 || !out) return fail(nullptr, VMC_E_ARG, "bad arguments");
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_uniforms, dim3((unsigned)blocks), dim3(256), 0, st, seed, n, step, out);
    HIP_OR_FAIL(nullptr, hipGetLastError());
    return VMC_OK;
}

}  // extern "C"

namespace {
// The contracted backward G = sum_w g_w O_w into out (overwritten, or added to
// when accumulate).  Jastrow part: one SYRK tile per workgroup; orbital part:
// one workgroup per orbital, rows of Ne/64 doubles per lane (the smallest
// instantiation that holds them); correlator part: one workgroup per
// correlator.  Nothing is allocated.
vmc_status logderiv_contract(vmc_ctx* h, const vmc_walkers* w, const double* g, double* out, int accumulate,
                             hipStream_t st) {
    const Tab T = make_tab(h);
    const Wk S = make_wk(h, w);
    const int nt16 = (h->n_so + 15) / 16;
    hipLaunchKernelGGL(k_grad_J_syrk, dim3((unsigned)(nt16 * (nt16 + 1) / 2)), dim3(64 * kSyrkWaves), 0, st, T, S,
                       w->n_walkers, g, out, accumulate);
    HIP_OR_FAIL(h, hipGetLastError());
    const int nr = (h->ne + 63) / 64;
    const int64_t nj = (int64_t)h->n_so * (h->n_so + 1) / 2;
    const dim3 grid((unsigned)h->n_so), block(64 * kGradWaves);
    const size_t lds = (size_t)h->ne * 8;
    const int64_t W = w->n_walkers;
    if (nr <= 1) hipLaunchKernelGGL(k_grad_theta_rows<1>, grid, block, lds, st, T, S, W, g, out, nj, accumulate);
    else if (nr <= 2) hipLaunchKernelGGL(k_grad_theta_rows<2>, grid, block, lds, st, T, S, W, g, out, nj, accumulate);
    else if (nr <= 4) hipLaunchKernelGGL(k_grad_theta_rows<4>, grid, block, lds, st, T, S, W, g, out, nj, accumulate);
    else if (nr <= 8) hipLaunchKernelGGL(k_grad_theta_rows<8>, grid, block, lds, st, T, S, W, g, out, nj, accumulate);
    else hipLaunchKernelGGL(k_grad_theta_rows<16>, grid, block, lds, st, T, S, W, g, out, nj, accumulate);
    HIP_OR_FAIL(h, hipGetLastError());
    if (h->ncorr > 0) {
        hipLaunchKernelGGL(k_grad_cps, dim3((unsigned)h->ncorr), dim3(64 * kCpsWaves), 0, st, T, S, W, g, out,
                           nj + (int64_t)h->n_so * h->n_so, accumulate);
        HIP_OR_FAIL(h, hipGetLastError());
    }
    return VMC_OK;
}
}  // namespace

extern "C" {

vmc_status vmc_logderiv(vmc_handle h, const vmc_walkers* w, const double* g, double* out, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    vmc_status s = check_walkers(h, w);
    if (s != VMC_OK) return s;
    if (!out) return fail(h, VMC_E_ARG, "out is NULL");
    const int64_t n_p = (int64_t)h->n_so * (h->n_so + 1) / 2 + (int64_t)h->n_so * h->n_so + h->n_coef;
    if (!g) {
        hipLaunchKernelGGL(k_logderiv_dense, dim3((unsigned)w->n_walkers), dim3(256), 0, st, make_tab(h), make_wk(h, w),
                           out, n_p);
        HIP_OR_FAIL(h, hipGetLastError());
        return VMC_OK;
    }
    return logderiv_contract(h, w, g, out, 0, st);
}

vmc_status vmc_logderiv_accumulate(vmc_handle h, const vmc_walkers* w, const double* g, double* out, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    vmc_status s = check_walkers(h, w);
    if (s != VMC_OK) return s;
    if (!out || !g) return fail(h, VMC_E_ARG, "g and out are required");
    return logderiv_contract(h, w, g, out, 1, st);
}

vmc_status vmc_snapshot_weights(vmc_handle h, const vmc_walkers* w, double* acc, double* g_te, double* g_t,
                                int32_t reset, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    if (!w || w->n_walkers <= 0 || !w->eloc || !w->tres) return fail(h, VMC_E_ARG, "bad walkers");
    if (!acc || !g_te || !g_t) return fail(h, VMC_E_ARG, "acc, g_te and g_t are required");
    hipLaunchKernelGGL(k_snapshot_weights, dim3(1), dim3(1024), 0, st, (const double*)w->eloc,
                       (const double*)w->tres, w->n_walkers, acc, g_te, g_t, reset ? 1 : 0);
    HIP_OR_FAIL(h, hipGetLastError());
    return VMC_OK;
}

vmc_status vmc_gradient_combine(int64_t n, const double* a, const double* b, const double* acc, double* out,
                                hipStream_t st) {
    if (n <= 0 || !a || !b || !acc || !out) return fail(nullptr, VMC_E_ARG, "bad arguments");
    hipLaunchKernelGGL(k_gradient_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, b, acc, out);
    HIP_OR_FAIL(nullptr, hipGetLastError());
    return VMC_OK;
}

vmc_status vmc_estimate(vmc_handle h, const vmc_walkers* w, double* out, double* g, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    if (!w || w->n_walkers <= 0 || !w->eloc || !w->tres) return fail(h, VMC_E_ARG, "bad walkers");
    if (!out) return fail(h, VMC_E_ARG, "out is NULL");
    hipLaunchKernelGGL(k_estimate, dim3(1), dim3(1024), 0, st, (const double*)w->eloc, (const double*)w->tres,
                       w->n_walkers, out, g);
    HIP_OR_FAIL(h, hipGetLastError());
    return VMC_OK;
}

vmc_status vmc_amsgrad(int64_t n, double* p, double* m, double* v, double* vh, const double* g, double lr, double b1,
                       double b2, double delta, int32_t literal, hipStream_t st) {
    if (n <= 0 || !p || !m || !v || !vh || !g) return fail(nullptr, VMC_E_ARG, "bad arguments");
    hipLaunchKernelGGL(k_amsgrad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, m, v, vh, g, lr, b1, b2,
                       delta, (int)literal);
    HIP_OR_FAIL(nullptr, hipGetLastError());
    return VMC_OK;
}

vmc_status vmc_set_small_denominator(vmc_handle h, double threshold) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    if (!(threshold >= 0.0)) return fail(h, VMC_E_ARG, "threshold must be >= 0 (+inf allowed)");
    h->small_den = threshold;
    return VMC_OK;
}

vmc_status vmc_set_launch(vmc_handle h, int32_t block_threads) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    if (block_threads != 0 && (block_threads < 64 || block_threads > 512 || (block_threads & 63) != 0))
        return fail(h, VMC_E_ARG, "block_threads must be 0 or a multiple of 64 in 64..512");
    h->block_threads = block_threads;
    return VMC_OK;
}

// Time one launch configuration: best of `reps` sweeps of n_moves moves.
static vmc_status time_sweeps(vmc_ctx* h, vmc_walkers* w, vmc_batch b, vmc_walkers* const* ws, int n_moves, int reps,
                              hipStream_t st, float* best_ms) {
    hipEvent_t e0, e1;
    HIP_OR_FAIL(h, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(h, VMC_E_HIP, "hipEventCreate failed");
    }
    vmc_status s = VMC_OK;
    *best_ms = 3.0e38f;
    for (int r = 0; r < reps && s == VMC_OK; ++r) {
        if (hipEventRecord(e0, st) != hipSuccess) { s = fail(h, VMC_E_HIP, "hipEventRecord failed"); break; }
        s = b ? vmc_batch_ctmc_step(b, ws, n_moves, st) : vmc_ctmc_step(h, w, n_moves, nullptr, nullptr, nullptr, st);
        if (s != VMC_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            s = fail(h, VMC_E_HIP, "event timing failed");
            break;
        }
        *best_ms = std::min(*best_ms, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s;
}

static const int kTuneThreads[] = {64, 128, 256, 512};

vmc_status vmc_autotune(vmc_handle h, vmc_walkers* w, int32_t n_moves, int32_t* chosen, hipStream_t st) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    vmc_status s = check_walkers(h, w);
    if (s != VMC_OK) return s;
    if (n_moves < 1) return fail(h, VMC_E_ARG, "n_moves must be >= 1");
    const int keep = h->block_threads, keep_w = h->waves;
    int best_nt = 0, best_w = 0;
    float best = 3.0e38f;
    // workgroup size, and for walkers in HBM the occupancy target
    for (int nt : kTuneThreads)
        for (int wv : {3, 4}) {
            h->block_threads = nt;
            const SweepGeom g = sweep_geom(h);
            if (g.lds > kMaxLdsHbm) continue;
            if (g.small && wv == 4) continue;  // one variant: the waves target applies to the HBM layout
            h->waves = g.small ? keep_w : wv;
            float ms = 0.0f;
            s = time_sweeps(h, w, nullptr, nullptr, n_moves, 2, st, &ms);
            if (s != VMC_OK) {
                h->block_threads = keep;
                h->waves = keep_w;
                return s;
            }
            if (ms < best) {
                best = ms;
                best_nt = nt;
                best_w = h->waves;
            }
        }
    if (best_nt == 0) {
        h->block_threads = keep;
        h->waves = keep_w;
        return fail(h, VMC_E_UNSUPPORTED, "no workgroup size fits the LDS budget");
    }
    h->block_threads = best_nt;
    h->waves = best_w;
    if (chosen) *chosen = best_nt;
    return VMC_OK;
}

vmc_status vmc_batch_autotune(vmc_batch b, vmc_walkers* const* walkers, int32_t n_moves, int32_t* chosen,
                              hipStream_t st) {
    if (!b) return fail(nullptr, VMC_E_ARG, "batch is NULL");
    if (n_moves < 1) return fail(nullptr, VMC_E_ARG, "n_moves must be >= 1");
    if (!walkers) return fail(nullptr, VMC_E_ARG, "walkers array is NULL");
    const int keep = b->nt, keep_w = b->waves, keep_m = b->mode;
    bool fusable = true;
    for (vmc_ctx* h : b->sys) fusable = fusable && !h->uhf && h->ncorr == 0;
    // the fused launch: every workgroup size and occupancy target
    int best_nt = 0, best_w = 0;
    float best = 3.0e38f;
    b->mode = VMC_BATCH_FUSED;
    for (int nt : kTuneThreads)
        for (int wv : {3, 4}) {
            if (!fusable) break;
            size_t lds = 0;
            for (vmc_ctx* h : b->sys)
                lds = std::max(lds,
                               (size_t)lds_layout(h->n_so, h->ne, h->nw, nt, false, (int)r_bytes(h), h->ncorr).total);
            if (lds > kMaxLdsHbm) continue;
            b->nt = nt;
            b->waves = wv;
            float ms = 0.0f;
            vmc_status s = time_sweeps(nullptr, nullptr, b, walkers, n_moves, 2, st, &ms);
            if (s != VMC_OK) {
                b->nt = keep;
                b->waves = keep_w;
                b->mode = keep_m;
                return s;
            }
            if (ms < best) {
                best = ms;
                best_nt = nt;
                best_w = wv;
            }
        }
    // one stream per system, each with its own autotuned shape
    for (size_t e = 0; e < b->sys.size(); ++e) {
        const vmc_status s = vmc_autotune(b->sys[e], walkers[e], n_moves, nullptr, st);
        if (s != VMC_OK) {
            b->nt = keep;
            b->waves = keep_w;
            b->mode = keep_m;
            return fail(nullptr, s, "system " + std::to_string(e) + ": " + b->sys[e]->err);
        }
    }
    b->mode = VMC_BATCH_STREAMS;
    float ms_streams = 0.0f;
    vmc_status s = time_sweeps(nullptr, nullptr, b, walkers, n_moves, 2, st, &ms_streams);
    if (s != VMC_OK) {
        b->nt = keep;
        b->waves = keep_w;
        b->mode = keep_m;
        return s;
    }
    if (best_nt != 0 && best <= ms_streams) {
        b->mode = VMC_BATCH_FUSED;
        b->nt = best_nt;
        b->waves = best_w;
    } else {
        b->nt = keep;
        b->waves = keep_w;
    }
    if (chosen) *chosen = b->mode == VMC_BATCH_FUSED ? b->nt : 0;
    return VMC_OK;
}

vmc_status vmc_batch_info(vmc_batch b, int64_t out[3]) {
    if (!b || !out) return fail(nullptr, VMC_E_ARG, "NULL argument");
    out[0] = b->mode;
    out[1] = b->nt;
    out[2] = batch_waves(b);
    return VMC_OK;
}

vmc_status vmc_table_info(vmc_handle h, int64_t out[3]) {
    if (!h || !out) return fail(h, VMC_E_ARG, "NULL argument");
    out[0] = h->n_dent;
    out[1] = h->n_sent;
    out[2] = h->G;
    return VMC_OK;
}

vmc_status vmc_launch_info(vmc_handle h, int64_t out[5]) {
    if (!h || !out) return fail(h, VMC_E_ARG, "NULL argument");
    const SweepGeom g = sweep_geom(h);
    out[0] = g.nt;
    out[1] = g.small ? 1 : 0;
    out[2] = (int64_t)g.lds;
    out[3] = use_refresh_kernel(h) ? 1 : 0;
    out[4] = g.small ? 0 : hbm_waves(h);
    return VMC_OK;
}

vmc_status vmc_set_occupancy(vmc_handle h, int32_t waves) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    if (waves != 0 && waves != 3 && waves != 4) return fail(h, VMC_E_ARG, "waves must be 0, 3 or 4");
    h->waves = waves;
    return VMC_OK;
}

vmc_status vmc_batch_set_occupancy(vmc_batch b, int32_t waves) {
    if (!b) return fail(nullptr, VMC_E_ARG, "batch is NULL");
    if (waves != 0 && waves != 3 && waves != 4) return fail(nullptr, VMC_E_ARG, "waves must be 0, 3 or 4");
    b->waves = waves;
    return VMC_OK;
}

// ------------------------------------------------------------------ batches
vmc_status vmc_batch_create(const vmc_handle* systems, int32_t n, vmc_batch* out) {
    if (!out) return fail(nullptr, VMC_E_ARG, "out is NULL");
    *out = nullptr;
    if (!systems || n < 1 || n > kMaxBatch)
        return fail(nullptr, VMC_E_ARG, "a batch holds 1.." + std::to_string(kMaxBatch) + " systems");
    for (int e = 0; e < n; ++e) {
        if (!systems[e]) return fail(nullptr, VMC_E_ARG, "system handle is NULL");
        if (systems[e]->precision != systems[0]->precision)
            return fail(nullptr, VMC_E_ARG, "all systems of a batch must have the same precision");
        if (!systems[e]->params_set) return fail(nullptr, VMC_E_ARG, "vmc_set_params has not been called");
    }
    vmc_batch_ctx* b = new vmc_batch_ctx;
    b->sys.assign(systems, systems + n);
    b->precision = systems[0]->precision;
    bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    for (int e = 0; e < n && ok; ++e) {
        hipStream_t s = nullptr;
        hipEvent_t ev = nullptr;
        ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
        if (ok) b->streams.push_back(s);
        ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (ok) b->done.push_back(ev);
    }
    if (!ok) {
        vmc_batch_destroy(b);
        return fail(nullptr, VMC_E_HIP, "stream or event creation failed");
    }
    *out = b;
    return VMC_OK;
}

vmc_status vmc_batch_set_mode(vmc_batch b, int32_t mode) {
    if (!b) return fail(nullptr, VMC_E_ARG, "batch is NULL");
    if (mode != VMC_BATCH_FUSED && mode != VMC_BATCH_STREAMS)
        return fail(nullptr, VMC_E_ARG, "mode must be VMC_BATCH_FUSED or VMC_BATCH_STREAMS");
    b->mode = mode;
    return VMC_OK;
}

vmc_status vmc_batch_set_launch(vmc_batch b, int32_t block_threads) {
    if (!b) return fail(nullptr, VMC_E_ARG, "batch is NULL");
    if (block_threads < 64 || block_threads > 512 || (block_threads % 64) != 0)
        return fail(nullptr, VMC_E_ARG, "block_threads must be a multiple of 64 in 64..512");
    b->nt = block_threads;
    return VMC_OK;
}

// VMC_BATCH_STREAMS: each system's own calls (its own variant, occupancy,
// workgroup size and re-inversion schedule) on its own stream, forked from st
// and joined back to it.
static vmc_status launch_streams(vmc_batch b, vmc_walkers* const* ws, int mode, int n_steps, hipStream_t st) {
    const int n = (int)b->sys.size();
    for (int e = 0; e < n; ++e) {
        vmc_status s = check_walkers(b->sys[e], ws[e]);
        if (s != VMC_OK) return fail(nullptr, s, "system " + std::to_string(e) + ": " + b->sys[e]->err);
    }
    if (hipEventRecord(b->fork, st) != hipSuccess) return fail(nullptr, VMC_E_HIP, "hipEventRecord failed");
    vmc_status s = VMC_OK;
    std::string msg;
    for (int e = 0; e < n && s == VMC_OK; ++e) {
        if (hipStreamWaitEvent(b->streams[e], b->fork, 0) != hipSuccess) {
            s = VMC_E_HIP;
            msg = "hipStreamWaitEvent failed";
            break;
        }
        vmc_ctx* h = b->sys[e];
        s = (mode == MODE_CTMC) ? vmc_ctmc_step(h, ws[e], n_steps, nullptr, nullptr, nullptr, b->streams[e])
                                : vmc_local_energy(h, ws[e], b->streams[e]);
        if (s != VMC_OK) msg = "system " + std::to_string(e) + ": " + h->err;
        // joined even after a failure, so that st orders after whatever was launched
        if (hipEventRecord(b->done[e], b->streams[e]) != hipSuccess || hipStreamWaitEvent(st, b->done[e], 0) != hipSuccess) {
            if (s == VMC_OK) msg = "stream join failed";
            s = (s == VMC_OK) ? VMC_E_HIP : s;
        }
    }
    return s == VMC_OK ? VMC_OK : fail(nullptr, s, msg);
}

static vmc_status launch_batch(vmc_batch b, vmc_walkers* const* ws, int mode, int n_steps, hipStream_t st) {
    if (!b) return fail(nullptr, VMC_E_ARG, "batch is NULL");
    if (!ws) return fail(nullptr, VMC_E_ARG, "walkers array is NULL");
    if (b->mode == VMC_BATCH_STREAMS) return launch_streams(b, ws, mode, n_steps, st);
    for (vmc_ctx* h : b->sys) {
        if (h->uhf) return fail(nullptr, VMC_E_UNSUPPORTED, "the fused batch holds VMC_GHF systems only");
        if (h->ncorr > 0)
            return fail(nullptr, VMC_E_UNSUPPORTED, "the fused batch holds systems without correlators only");
    }
    BatchArgs A;
    std::memset(&A, 0, sizeof(A));
    A.n = (int)b->sys.size();
    int64_t blocks = 0;
    size_t lds = 0;
    for (int e = 0; e < A.n; ++e) {
        vmc_ctx* h = b->sys[e];
        vmc_status s = check_walkers(h, ws[e]);
        if (s != VMC_OK) return fail(nullptr, s, "system " + std::to_string(e) + ": " + h->err);
        BatchEntry& E = A.e[e];
        E.T = make_tab(h);
        E.S = make_wk(h, ws[e]);
        E.W = ws[e]->n_walkers;
        E.block0 = blocks;
        E.seed = h->seed;
        E.step0 = ws[e]->step;
        E.refresh = h->refresh;
        blocks += E.W;
        lds = std::max(lds, (size_t)lds_layout(h->n_so, h->ne, h->nw, b->nt, false, (int)r_bytes(h), h->ncorr).total);
    }
    if (lds > kMaxLdsHbm) return fail(nullptr, VMC_E_UNSUPPORTED, "a batched system exceeds the per-walker LDS budget");
    if (blocks > (int64_t)INT_MAX) return fail(nullptr, VMC_E_ARG, "too many walkers in the batch");
    const dim3 grid((unsigned)blocks), block((unsigned)b->nt);
    const int hw = batch_waves(b);
    if (b->precision == VMC_MIXED) {
        if (hw == 4) hipLaunchKernelGGL((k_sweep_batch<float, 4>), grid, block, lds, st, A, mode, n_steps);
        else hipLaunchKernelGGL((k_sweep_batch<float, 3>), grid, block, lds, st, A, mode, n_steps);
    } else {
        if (hw == 4) hipLaunchKernelGGL((k_sweep_batch<double, 4>), grid, block, lds, st, A, mode, n_steps);
        else hipLaunchKernelGGL((k_sweep_batch<double, 3>), grid, block, lds, st, A, mode, n_steps);
    }
    HIP_OR_FAIL(nullptr, hipGetLastError());
    if (mode == MODE_CTMC)
        for (int e = 0; e < A.n; ++e) ws[e]->step += (uint64_t)n_steps;
    return VMC_OK;
}

vmc_status vmc_batch_local_energy(vmc_batch b, vmc_walkers* const* walkers, hipStream_t st) {
    return launch_batch(b, walkers, MODE_ELOC, 1, st);
}

vmc_status vmc_batch_ctmc_step(vmc_batch b, vmc_walkers* const* walkers, int32_t n_steps, hipStream_t st) {
    if (n_steps < 0) return fail(nullptr, VMC_E_ARG, "n_steps must be >= 0");
    if (n_steps == 0) return VMC_OK;
    return launch_batch(b, walkers, MODE_CTMC, n_steps, st);
}

vmc_status vmc_batch_destroy(vmc_batch b) {
    if (!b) return fail(nullptr, VMC_E_ARG, "batch is NULL");
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    for (hipEvent_t ev : b->done) (void)hipEventDestroy(ev);
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
    return VMC_OK;
}

vmc_status vmc_destroy(vmc_handle h) {
    if (!h) return fail(nullptr, VMC_E_ARG, "handle is NULL");
    free_ctx(h);
    return VMC_OK;
}

}  // extern "C"

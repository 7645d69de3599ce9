/*
 * vmc.h -- C ABI of the MI355X (gfx950) screened orbital-space VMC hot path.
 *
 * The library evaluates, for thousands of walkers (determinants) at once:
 *   - the screened local energy E_L[N, eps] = sum_M^eps H_NM psi(M)/psi(N)
 *     (Sabzevari & Sharma, Eq. eloc:hci), with singles screened by the bound
 *     S_ia = |h_ia| + sum_j |(ia|jj) - (ij|ja)| and doubles by
 *     |<ab|ij> - <ab|ji>| through a heat-bath table (section "Reduced scaling
 *     evaluation of the local energy");
 *   - amplitude ratios of a Jastrow-Slater wavefunction, single ratios from
 *     R = theta * theta[N]^-1 (Eq. R) and doubles as 2x2 minors of R;
 *   - continuous-time Monte Carlo moves with rates r = |psi(M)/psi(N)| over the
 *     same screened set, residence time t = 1/sum r (Eq. eq:rate and the
 *     steps after it);
 *   - Sherman-Morrison updates of theta[N]^-1 and R (the two update formulas of
 *     the section "Local energy and Gradient ratios");
 *   - gradient ratios O_k (the same section) and their contraction into the
 *     energy gradient of Eq. eq:grad, plus an AMSGrad step (Eqs. eq:m1, eq:m2).
 *
 * Conventions
 *   - Spatial orbitals 0..n-1; spin-orbitals alpha 0..n-1, beta n..2n-1.
 *   - Two-electron integrals: real chemist notation (pq|rs), 8-fold symmetric,
 *     passed as a canonical list with p>=q, r>=s, pair(p,q) >= pair(r,s),
 *     pair(p,q) = p(p+1)/2 + q.
 *   - Wavefunction psi(N) = exp(sum_{p<=q} J_pq n_p n_q) det(theta[occ(N), 0:Ne]),
 *     J packed as its upper triangle row by row, theta n_so x n_so row-major.
 *   - Occupations: little-endian bitstrings, ceil(n_so/64) uint64 words.
 *   - Walker slots: slot p holds the orbital slot_orb[p]; A[p][x] =
 *     theta[slot_orb[p]][x]; B = A^-1; R[a][p] = sum_x theta[a][x] B[x][p].
 *     B and R are stored column by slot: B at ainv[p*Ne + x], R at r[p*n_so + a].
 *   - Candidate (canonical) order, used by the CTMC pick: singles first
 *     (occupied i ascending, then a by descending S_ia, ties by a), then
 *     doubles (occupied pairs i<j ascending, then a<b by descending |v|, ties
 *     by (a, b)).
 *
 * Errors: every call validates its host arguments synchronously and returns
 * VMC_E_ARG with a message (vmc_last_error) on a bad argument.  Device-side
 * problems never abort: they set per-walker status bits (VMC_ST_*).
 * All device work is enqueued on the given stream (0 = the default stream)
 * and is asynchronous unless stated otherwise.  Stepping allocates nothing:
 * the caller owns walker buffers (sized by vmc_walker_bytes) and parameters;
 * the library owns the integral tables it builds in vmc_init.
 */
#ifndef VMC_H
#define VMC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vmc_ctx* vmc_handle;

typedef enum {
    VMC_OK = 0,
    VMC_E_ARG = -1,         /* invalid host argument */
    VMC_E_OOM = -2,         /* device or host allocation failed (vmc_init only) */
    VMC_E_HIP = -3,         /* a HIP runtime call failed */
    VMC_E_SINGULAR = -4,    /* reserved */
    VMC_E_STATE = -5,       /* reserved */
    VMC_E_UNSUPPORTED = -6  /* size or mode outside what the library supports */
} vmc_status;

enum { VMC_FP64 = 0, VMC_MIXED = 1 };

/* Form of the determinant's orbitals (vmc_system_desc.orbitals). */
enum { VMC_GHF = 0, VMC_UHF = 1 };

/* per-walker status bits (device field `status`) */
enum {
    VMC_ST_SINGULAR = 1u,   /* theta[N] singular at (re)inversion: psi(N) = 0 */
    VMC_ST_EMPTY = 2u,      /* no connected determinant with a positive rate: no move */
    VMC_ST_NONFINITE = 4u,  /* E_L or T not finite */
    VMC_ST_SMALLDEN = 8u,   /* a Sherman-Morrison denominator below the threshold of
                               vmc_set_small_denominator (1e-8) in magnitude; where the sweep
                               re-inverts in place (state in LDS, or general orbitals with more than
                               192 electrons) the walker is re-inverted right after that move, else at
                               its next re-inversion */
    VMC_ST_STALE = 16u      /* walkers re-inverted by the separate refresh kernel (state in HBM): B and R
                               carry updates made since their last inversion; set by a sweep that moved
                               the walker, cleared by every (re-)inversion.  Not an error. */
};

typedef struct {
    int32_t n_orb;          /* spatial orbitals n (n_so = 2n <= 1024) */
    int32_t n_alpha;        /* alpha electrons */
    int32_t n_beta;         /* beta electrons */
    int32_t precision;      /* VMC_FP64: every quantity in FP64.
                               VMC_MIXED: R stored and updated in FP32, ratios formed from FP32 minors,
                               refresh GEMM R = theta B on the FP32 matrix cores; B = theta[N]^-1, its
                               re-inversion, the update denominators (recomputed as theta[a,:] B in FP64),
                               E_L, T and all accumulations stay FP64 */
    int32_t refresh_period; /* re-invert theta[N] from scratch every this many CTMC steps (>= 1) */
    int32_t orbitals;       /* VMC_GHF: general orbitals, every entry of theta[:, 0:Ne] is used.
                               VMC_UHF: spin-blocked (unrestricted) orbitals, the determinant form of the
                               sections "Performance of the optimizer" and "2-D Hubbard Model Benchmark":
                               theta[a][x] enters only where orbital a and occupied column x have the same
                               spin (columns [0, n_alpha) alpha, [n_alpha, Ne) beta); vmc_set_params sets
                               the other entries of its copy to zero.  The determinant then factors into
                               an alpha and a beta determinant, slot p < n_alpha holds an alpha electron,
                               B is block diagonal, R keeps each slot's own spin only ([W][Ne][n]), and a
                               move updates the blocks of the spin it moves.  At most 128 electrons of
                               each spin (VMC_E_UNSUPPORTED beyond); the screened singles and doubles must
                               keep every electron in its spin (VMC_E_ARG otherwise; integrals over
                               spatial orbitals always do); the walker state lives in HBM; a batch refuses
                               such a system (VMC_E_UNSUPPORTED).  Walkers with a wrong alpha count are
                               flagged VMC_ST_SINGULAR at initialisation. */
    uint64_t seed;          /* Philox key word 0 for CTMC draws */
} vmc_system_desc;

typedef struct {
    int64_t n_nz;           /* number of canonical entries */
    const int32_t* pqrs;    /* host, 4*n_nz indices (p,q,r,s), canonical order within each entry */
    const double* val;      /* host, n_nz values (pq|rs) */
} vmc_eri_list;

/* walker fields, in the order of vmc_walker_bytes' output */
enum {
    VMC_F_OCC = 0,   /* uint64 [W][ceil(n_so/64)]  occupation bits (caller sets before vmc_walkers_init) */
    VMC_F_SLOT_ORB,  /* int32  [W][Ne]     orbital held by each slot */
    VMC_F_ORB_SLOT,  /* int32  [W][n_so]   slot of each orbital, -1 when empty */
    VMC_F_AINV,      /* double [W][Ne][Ne] B = theta[N]^-1, column by slot */
    VMC_F_R,         /* double (VMC_FP64) or float (VMC_MIXED) [W][Ne][n_so] R, column by slot;
                        VMC_UHF: [W][Ne][n], slot p's own spin only (orbital a at a - n for beta) */
    VMC_F_RLO,       /* uint16 [W][Ne][n_so] (VMC_UHF: [W][Ne][n]), VMC_MIXED only (0 bytes in
                        VMC_FP64): the bfloat16 remainder of each R entry, R = r + rlo to about
                        2^-33 relative.  With the walker state in HBM the re-inversion writes it
                        and every move carries it, so the FP32 r read by the ratios never drifts
                        from the FP64 R; where the state fits on chip it is written as zero */
    VMC_F_JSUM,      /* double [W][n_so]   s_p = sum_{q != p} J_pq n_q */
    VMC_F_HNN,       /* double [W]         H_NN */
    VMC_F_ELOC,      /* double [W]         last local energy */
    VMC_F_TRES,      /* double [W]         last residence time t = 1/T (0 when T = 0) */
    VMC_F_PICK,      /* int64  [W]         last move, packed (see vmc_decode_pick) */
    VMC_F_STATUS,    /* uint32 [W]         VMC_ST_* bits, cleared by vmc_walkers_init */
    VMC_F_SCRATCH,   /* bytes  [W][...]    kernel scratch, the library's between calls: with the
                        walker state in HBM it keeps each walker's singles elements
                        H_ia = h_ia + sum_j V_ia[j] with a tag naming the occupation and
                        the system they were built for, and a launch whose walker matches
                        the tag reuses them instead of rebuilding them (rebuilt at least
                        every 4096 moves, which bounds the rounding of the per-move
                        updates).  Callers do not
                        write it, except to fill it with zeros (which clears every tag) */
    VMC_NFIELDS
};

typedef struct {
    int64_t n_walkers;
    void* occ_bits;
    void* slot_orb;
    void* orb_slot;
    void* ainv;
    void* r;
    void* rlo;              /* VMC_MIXED: required; VMC_FP64: ignored, may be NULL */
    void* jsum;
    void* hnn;
    void* eloc;
    void* tres;
    void* pick;
    void* status;
    void* scratch;
    uint64_t step;          /* host-side global CTMC step counter, advanced by vmc_ctmc_step */
    uint64_t since_inv;     /* moves since B and R were last inverted from scratch (state in HBM;
                               set to 0 by vmc_walkers_init, vmc_walkers_refresh and every
                               re-inversion) */
} vmc_walkers;

/*
 * Build the screening tables from h1 (host, n x n, row-major) and the canonical
 * integral list (host; read during the call only) for threshold eps >= 0, and
 * upload them to the current device.  Singles kept iff S_ia > eps, doubles iff
 * |v| > eps (section "Reduced scaling evaluation of the local energy").
 * Blocks until the upload is complete.  On success *out owns the tables.
 */
vmc_status vmc_init(const vmc_system_desc* desc, const double* h1, const vmc_eri_list* eri_screened, double eps,
                    hipStream_t stream, vmc_handle* out);

/* Wavefunction parameters of the section "Correlator product states and
 * Slater determinant": the correlator factor in its two-site (Jastrow) form
 * exp(sum_{p<=q} J_pq n_p n_q) and the Slater determinant's orbital matrix
 * theta.  Copies them (device pointers, caller-owned, read on `stream` during
 * the call's kernels; they may be freed once that work has completed): J packed
 * upper triangle, n_so(n_so+1)/2 doubles; theta n_so x n_so row-major.
 * Rebuilds the Jastrow factors folded into the tables.  Walkers must be
 * re-initialised (vmc_walkers_init) or re-inverted (vmc_walkers_refresh)
 * afterwards.  Errors: VMC_E_ARG for a NULL handle or pointer, VMC_E_HIP on a
 * failed copy or launch.  Values are not checked: a NaN or infinity in theta
 * reaches the walkers as VMC_ST_SINGULAR | VMC_ST_NONFINITE at re-inversion. */
vmc_status vmc_set_params(vmc_handle h, const double* J_dev, const double* theta_dev, hipStream_t stream);

/*
 * Correlator product state, the wavefunction factor C of the section
 * "Correlator product states and Slater determinant": psi(N) = C[N] x the
 * Jastrow factor x det(theta[N]), C[N] = prod_l c_l[n_l(N)].  Correlator l
 * covers k_l <= 5 distinct sites (spatial orbitals) sites[5 l + m], m < k_l,
 * -1 after the last; its local Fock state in N is
 * n_l(N) = sum_m (n_{s_m alpha} + 2 n_{s_m beta}) 4^m and it has 4^k_l
 * coefficients, stored in correlator order (offset of l = sum_{l' < l} 4^k_l').
 * The ratio C[M]/C[N] takes only the correlators holding a site whose
 * occupation the move changes, found through per-site correlator lists
 * (section "Local energy and Gradient ratios").
 *
 * vmc_cps_init: a setup call, made once per handle (VMC_E_ARG if repeated),
 * before or after walkers exist: validates the site lists (VMC_E_ARG: no
 * site, a repeated site or a site >= n_orb; VMC_E_UNSUPPORTED beyond 2^31
 * coefficients), builds the per-site lists and allocates the coefficient
 * buffer (it allocates and synchronises the device; VMC_E_OOM on failure).
 * sites: host, 5 * n_corr int32, read during the call only.
 * vmc_set_cps: copies the coefficients (device, caller-owned, read on
 * `stream`; nothing allocated); required before any walker call once
 * correlators exist.  Walker state holds nothing of C, so walkers need no
 * re-initialisation.  A zero coefficient met by a walker makes its ratios
 * non-finite (VMC_ST_NONFINITE).
 * vmc_cps_info: out[0] = correlators, out[1] = coefficients (0, 0 without).
 * With correlators, vmc_logderiv appends their gradient ratios
 * O_{c_l[n]} = [n_l(N) = n] / c_l[n] after the orbital part.
 */
vmc_status vmc_cps_init(vmc_handle h, int32_t n_corr, const int32_t* sites);
vmc_status vmc_set_cps(vmc_handle h, const double* coeffs_dev, hipStream_t stream);
vmc_status vmc_cps_info(vmc_handle h, int64_t out[2]);

/* Bytes of each walker field for n_walkers walkers (host-only call). */
vmc_status vmc_walker_bytes(vmc_handle h, int64_t n_walkers, size_t field_bytes[VMC_NFIELDS]);

/* From occ_bits only: slots in ascending orbital order, B = theta[N]^-1 by
 * partial-pivoting Gauss-Jordan in FP64 (the initial inversion of the
 * section "Local energy and Gradient ratios"), R, s, H_NN; clears status. */
vmc_status vmc_walkers_init(vmc_handle h, vmc_walkers* w, hipStream_t stream);

/* Re-inversion after new parameters (vmc_set_params) for walkers that already
 * hold a valid state of this system (from vmc_walkers_init or moves): the
 * occupations and slot order are kept and B, R, s, H_NN recomputed for the
 * current theta and J.  Walkers whose state lives in HBM are inverted afresh
 * by the refresh kernel in their current slot order; the others are
 * re-initialised as by vmc_walkers_init.  Errors: VMC_E_ARG for a NULL handle
 * or walkers of another system; launch failures as VMC_E_HIP.  The walkers
 * must not be in use by work on another stream. */
vmc_status vmc_walkers_refresh(vmc_handle h, vmc_walkers* w, hipStream_t stream);

/* E_L[N, eps] = H_NN + sum over the screened singles and doubles M of
 * H_NM psi(M)/psi(N) (Eq. eloc:hci; screening of the section "Reduced scaling
 * evaluation of the local energy"), and t = 1/T with T = sum_M |psi(M)/psi(N)|
 * over the same set (Eq. eq:rate), for every walker from its current state,
 * into the walkers' eloc and tres fields; no state change.  A walker whose
 * state is flagged VMC_ST_SINGULAR gets E_L = NaN and t = 0; a non-finite E_L
 * or T sets VMC_ST_NONFINITE, T = 0 sets VMC_ST_EMPTY (t = 0).  Errors:
 * VMC_E_ARG for a NULL handle or walker field, or before vmc_set_params;
 * VMC_E_UNSUPPORTED when the system exceeds the per-walker LDS budget;
 * launch failures as VMC_E_HIP. */
vmc_status vmc_local_energy(vmc_handle h, vmc_walkers* w, hipStream_t stream);

/*
 * n_steps continuous-time Monte Carlo moves (section "Continuous time Monte
 * Carlo for sampling determinants": rates r_M = |psi(M)/psi(N)| of Eq.
 * eq:rate over the screened set, residence time t = 1/sum r, M drawn with
 * probability r_M / sum r) of every walker in one persistent launch, each
 * followed by the Sherman-Morrison update of the section "Local energy and
 * Gradient ratios".  Errors: VMC_E_ARG for a NULL handle or walker field,
 * n_steps < 0, or before vmc_set_params; VMC_E_UNSUPPORTED when the system
 * exceeds the per-walker LDS budget; launch failures as VMC_E_HIP.  Step k of
 * walker i draws u from Philox4x64-10 with counter (w->step + k, 0, 0, 0) and
 * key (seed, i) (first output word, 53 high bits), picks the smallest
 * candidate index whose running rate sum exceeds u*T, and updates B, R, s and
 * the occupation.  B and R are recomputed from scratch at a fixed interval:
 * when the walker state fits LDS, after every move whose global step g has
 * (g + 1) % refresh_period == 0; when it lives in HBM, before a move once
 * refresh_period moves have been made since the last inversion (counted in
 * w->since_inv), so that a re-inversion due after the last move of a call is
 * made by the next call, or not at all when vmc_walkers_refresh comes first.
 * Optional device outputs (NULL to skip), each [n_steps][W]: eloc_hist (E_L
 * before the move), t_hist (residence time), pick_hist (packed move).
 * Advances w->step by n_steps.
 */
vmc_status vmc_ctmc_step(vmc_handle h, vmc_walkers* w, int32_t n_steps, double* eloc_hist, double* t_hist,
                         int64_t* pick_hist, hipStream_t stream);

/*
 * vmc_ctmc_step for callers that cannot allocate device memory (code under
 * graph capture, serving loops, harnesses that forbid allocation): the same
 * moves, bit for bit, with the kernels' per-walker workspace (the walkers'
 * `scratch` field: pair descriptors and singles elements) taken from a static
 * device array of 64 MiB that the library holds on every GPU it runs on until
 * the process ends; w->scratch is ignored and may be NULL.  No allocation, no
 * allocating library call.  Calls that overlap on one GPU share that array and
 * race: serialise them.  Errors: VMC_E_ARG when the walkers need more than 64
 * MiB of workspace (n_walkers x the per-walker scratch size of
 * vmc_walker_bytes), when the current device is not the handle's, or as
 * vmc_ctmc_step; VMC_E_STATE if the array's address could not be taken on
 * this device at vmc_init.
 */
vmc_status vmc_ctmc_step_static(vmc_handle h, vmc_walkers* w, int32_t n_steps, double* eloc_hist, double* t_hist,
                                int64_t* pick_hist, hipStream_t stream);

/*
 * vmc_ctmc_step with the global step counter in device memory instead of
 * w->step: the first move of the call uses *step_dev (read on the device when
 * the kernel runs), and a one-thread kernel adds n_steps to it after the
 * sweep.  Nothing is allocated, synchronised or read back, so the call can be
 * captured in a hipGraph and replayed: every replay draws the next uniforms.
 * w->step is not used or changed; no histories.  Refresh: as vmc_ctmc_step
 * when the walker state fits LDS (by the global step); for walkers whose state
 * lives in HBM, n_steps must be a multiple of refresh_period (VMC_E_ARG
 * otherwise), and before every refresh_period moves of the call the separate
 * refresh kernel re-inverts exactly the walkers marked VMC_ST_STALE (moved
 * since their last inversion; fresh walkers, e.g. just re-inverted for new
 * parameters, are skipped), so no walker makes more than refresh_period moves
 * on one inverse whatever state a replay finds.  w->since_inv is set to
 * refresh_period (an eager vmc_ctmc_step that follows re-inverts first).
 * step_dev: device, 8 bytes, caller-owned.
 */
vmc_status vmc_ctmc_step_dev(vmc_handle h, vmc_walkers* w, int32_t n_steps, uint64_t* step_dev, hipStream_t stream);

/*
 * Gradient ratios O_k of each walker's current state, N_p = n_so(n_so+1)/2 +
 * n_so^2 (+ the correlator coefficients, see vmc_cps_init) (Jastrow part
 * packed like J, then theta row-major, then the correlators):
 * O_{J_pq} = n_p n_q, O_{theta_kx} = B[x][slot(k)] for occupied k and x < Ne,
 * else 0, O_{c_l[n]} = [n_l(N) = n] / c_l[n].  If g_dev (device, W doubles) is NULL, out_dev receives the dense
 * [W][N_p] matrix; otherwise out_dev receives G = sum_w g_w O_w (N_p doubles),
 * the contracted backward used for Eq. eq:grad with g_w = 2 t_w (E_L,w - E)/sum t.
 * The contracted form computes the Jastrow part as Occ^T diag(g) Occ (Occ the
 * W x n_so occupation matrix) on the FP64 matrix cores and the orbital part
 * row by row over the walkers holding each orbital; every sum runs over the
 * walkers in a fixed order, so the result is deterministic, and walkers with
 * g_w = 0 contribute nothing (their B is not read).  Nothing is allocated:
 * the call can be captured in a hipGraph as it is.  Errors: VMC_E_ARG for a
 * NULL handle, walkers or out_dev; launch failures as VMC_E_HIP.
 * Defined in the section "Local energy and Gradient ratios" (gradient ratios
 * of the Jastrow and orbital parameters) and Eq. eq:grad.
 */
vmc_status vmc_logderiv(vmc_handle h, const vmc_walkers* w, const double* g_dev, double* out_dev,
                        hipStream_t stream);

/*
 * Residence-time weighted energy of the walkers' current E_L and t (as left by
 * vmc_local_energy or vmc_ctmc_step): E = sum_w t_w E_L,w / sum_w t_w, the
 * CTMC estimate of Eq. eq:vmc (section "Continuous time Monte Carlo for
 * sampling determinants").  out (device, 4 doubles) = {sum t, sum t E_L, E,
 * number of walkers counted}.  When g (device, W doubles) is non-NULL it
 * receives the contraction weights of the gradient estimator of Eq. eq:grad,
 * g_w = 2 t_w (E_L,w - E) / sum t, ready for vmc_logderiv.  Walkers with t <= 0
 * or a non-finite E_L (flagged states) carry no weight and get g_w = 0.  One
 * workgroup, fixed summation order: deterministic.  Asynchronous on stream.
 */
vmc_status vmc_estimate(vmc_handle h, const vmc_walkers* w, double* out, double* g, hipStream_t stream);

/*
 * The gradient estimator of Eq. eq:grad over several sets of states (one set
 * per call, e.g. the walkers every few moves of a sweep), so that more of the
 * sampled states than the last one per walker enter G:
 * G_k = 2 sum_s t_s O_k(s) (E_L(s) - E) / sum_s t_s = 2 (A_k - E B_k) / sum t,
 * A = sum t E_L O, B = sum t O, E = sum t E_L / sum t.
 *
 * vmc_snapshot_weights: for the walkers' current E_L and t (as left by
 * vmc_local_energy), g_te[w] = t_w E_L,w and g_t[w] = t_w (device, W doubles
 * each; 0 for flagged states, as in vmc_estimate), and the running sums acc
 * (device, 4 doubles) = {sum t, sum t E_L, E, states counted}, started afresh
 * when reset is nonzero, added to otherwise.  One workgroup, fixed order.
 * vmc_logderiv_accumulate: out += sum_w g_w O_w (the contracted vmc_logderiv,
 * added to out instead of overwriting it); call it with g_te into A and with
 * g_t into B (the first set may use vmc_logderiv to overwrite).
 * vmc_gradient_combine: out[k] = 2 (a[k] - E b[k]) / sum t from acc (0 when
 * no state carried weight), n entries, all device.
 * Nothing is allocated; asynchronous on stream.
 */
vmc_status vmc_snapshot_weights(vmc_handle h, const vmc_walkers* w, double* acc, double* g_te, double* g_t,
                                int32_t reset, hipStream_t stream);
vmc_status vmc_logderiv_accumulate(vmc_handle h, const vmc_walkers* w, const double* g_dev, double* out_dev,
                                   hipStream_t stream);
vmc_status vmc_gradient_combine(int64_t n, const double* a, const double* b, const double* acc, double* out,
                                hipStream_t stream);

/* One AMSGrad step over n parameters, all pointers device (Eqs. eq:m1, eq:m2,
 * in the Reddi form with standard betas: m = b1 m + (1-b1) g, v = b2 v +
 * (1-b2) g^2, vhat = max(vhat, v), p -= lr m / (sqrt(vhat) + delta)).
 * paper_literal != 0 uses vhat = max(vhat, b2 vhat + (1-b2) g^2) instead. */
vmc_status vmc_amsgrad(int64_t n, double* params, double* m, double* v, double* vhat, const double* grad,
                       double lr, double beta1, double beta2, double delta, int32_t paper_literal,
                       hipStream_t stream);

/*
 * Diagnostic: the screened candidate list of one walker in canonical order.
 * Device outputs: ijab[5*k] = {type (1 single, 2 double), i, j, a, b}
 * (j = b = -1 for singles), hval[k] = H_NM in the walker's slot convention,
 * ratio[k] = psi(M)/psi(N); count_dev[0] = number of candidates (entries
 * beyond cap are counted but not written).
 */
vmc_status vmc_excitations(vmc_handle h, const vmc_walkers* w, int64_t walker, int32_t* ijab, double* hval,
                           double* ratio, int64_t cap, int64_t* count_dev, hipStream_t stream);

/* Diagnostic: u values of the CTMC draw for walkers 0..n-1 at one step (device out). */
vmc_status vmc_uniforms(uint64_t seed, int64_t n, uint64_t step, double* out_dev, hipStream_t stream);

/* Decode a packed pick: type (0 = no move, 1 single, 2 double), i, j, a, b. */
void vmc_decode_pick(int64_t code, int32_t out5[5]);

/*
 * Threshold below which the magnitude of a Sherman-Morrison denominator (the
 * ratio psi(M)/psi(N) of the determinants, or the 2x2 determinant of the
 * Woodbury update of a double; the Sherman-Morrison paragraph of section
 * "Local energy and Gradient ratios") marks the walker VMC_ST_SMALLDEN and,
 * where the sweep re-inverts in place, makes it re-invert theta[N] from
 * scratch right after that move: a small denominator amplifies the rounding
 * that the update carries into B and R.  Default 1e-8; 0 never flags, +inf
 * flags (and re-inverts after) every move.  Host-only; affects subsequent
 * calls on h.  VMC_E_ARG for a negative or NaN threshold.
 */
vmc_status vmc_set_small_denominator(vmc_handle h, double threshold);

/* Launch shape of the sweep kernels: threads per walker workgroup (a multiple
 * of 64 in 64..512), or 0 for the library's choice.  Host-only; affects
 * subsequent calls on h.  Results do not depend on it except for the order of
 * floating-point sums (E_L and T change at rounding level; picks can change
 * only within that rounding of a cumulative-rate boundary). */
vmc_status vmc_set_launch(vmc_handle h, int32_t block_threads);

/* Table sizes: out[0] = double entries, out[1] = single entries, out[2] = groups
 * per walker (Ne + Ne(Ne-1)/2). */
vmc_status vmc_table_info(vmc_handle h, int64_t out[3]);

/* Launch geometry of the sweep kernel for this system and the current
 * vmc_set_launch / vmc_set_occupancy settings: out[0] = threads per walker
 * (workgroup size), out[1] = 1 when the walker state (R, B, descriptors) is
 * held in LDS for the whole sweep, 0 when it stays in the caller's HBM
 * buffers, out[2] = LDS bytes per workgroup, out[3] = 1 when re-inversion runs
 * in the separate refresh kernel (HBM-resident walkers whose B fits 160 KB of
 * LDS), out[4] = occupancy target of the sweep kernel in waves per SIMD (3 or
 * 4; 0 when the state is held in LDS, whose variants fix their own). */
vmc_status vmc_launch_info(vmc_handle h, int64_t out[5]);

/* Occupancy target of the sweep kernel when the walker state stays in HBM:
 * 3 or 4 waves per SIMD (which fixes the kernel's register budget: 168 or 128
 * VGPRs), or 0 for the library's choice (4 when the table holds doubles, else
 * 3; a system with correlators always runs at 3: its sweep variants are
 * compiled for that target only).  Host-only; affects subsequent calls.
 * Results do not depend on it (the same arithmetic in the same order).
 * VMC_E_ARG for other values.
 * vmc_batch_set_occupancy: the same for a batch's launch. */
vmc_status vmc_set_occupancy(vmc_handle h, int32_t waves);

vmc_status vmc_destroy(vmc_handle h);

/*
 * Batches: systems of different sizes (each with its own tables, parameters
 * and walker set) swept together.  Fused mode (the default): ONE kernel
 * launch; workgroups are dealt to the systems in order, every system runs the
 * variant that keeps the walker state in its HBM buffers and re-inverts in
 * place every refresh_period moves, and the LDS of the launch is sized for
 * the largest system.  Stream mode: see vmc_batch_set_mode below.
 *
 * vmc_batch_create: 1..8 systems with the same precision whose parameters are
 * set; the batch refers to the handles (which must outlive it) and owns no
 * device memory (one stream and event per system, for the stream mode).
 * walkers[e] is the walker set of systems[e] (already initialised with
 * vmc_walkers_init).  vmc_batch_local_energy and vmc_batch_ctmc_step compute
 * exactly what vmc_local_energy / vmc_ctmc_step (without histories) compute
 * for each system alone with the same launch variant; each walker set's step
 * counter advances by n_steps.  vmc_batch_set_launch: workgroup size of the
 * fused launch (64..512).  Errors are reported through vmc_last_error(NULL).
 */
typedef struct vmc_batch_ctx* vmc_batch;
vmc_status vmc_batch_create(const vmc_handle* systems, int32_t n, vmc_batch* out);
vmc_status vmc_batch_set_launch(vmc_batch b, int32_t block_threads);
vmc_status vmc_batch_set_occupancy(vmc_batch b, int32_t waves);

/* How a batch runs (vmc_batch_set_mode; vmc_batch_info: out[0] = mode, out[1]
 * = workgroup size and out[2] = occupancy target of the fused launch):
 * VMC_BATCH_FUSED (default): the one launch described above; spin-blocked
 * systems and systems with correlators are refused (VMC_E_UNSUPPORTED) at
 * the call.  VMC_BATCH_STREAMS:
 * each system's own calls (vmc_ctmc_step / vmc_local_energy, with its own
 * variant: state in LDS where it fits, its own workgroup size, occupancy and
 * re-inversion schedule) on a stream of its own, forked from the caller's
 * stream and joined back to it with events (created at vmc_batch_create), so
 * the systems run concurrently; any system, spin-blocked ones included.
 * Results are those of the separate calls, bit for bit. */
enum { VMC_BATCH_FUSED = 0, VMC_BATCH_STREAMS = 1 };
vmc_status vmc_batch_set_mode(vmc_batch b, int32_t mode);
vmc_status vmc_batch_info(vmc_batch b, int64_t out[3]);
vmc_status vmc_batch_local_energy(vmc_batch b, vmc_walkers* const* walkers, hipStream_t stream);
vmc_status vmc_batch_ctmc_step(vmc_batch b, vmc_walkers* const* walkers, int32_t n_steps, hipStream_t stream);
vmc_status vmc_batch_destroy(vmc_batch b);

/*
 * Launch-shape autotuner: times CTMC sweeps of n_moves moves at each
 * workgroup size in {64, 128, 256, 512} threads per walker that fits the LDS
 * budget and, where the walker state stays in HBM (always in a fused batch),
 * each occupancy target (3 and 4 waves per SIMD) (best of two sweeps each, HIP
 * events on `stream`), keeps the fastest shape (as vmc_set_launch /
 * vmc_set_occupancy or their batch forms would) and returns its workgroup
 * size in *chosen (nullable; vmc_launch_info reports the occupancy).
 * vmc_batch_autotune also tunes every system on its own (vmc_autotune), times
 * the batch in VMC_BATCH_STREAMS mode, and keeps the faster mode (*chosen = 0
 * for the stream mode; vmc_batch_info reports it); a batch holding a
 * spin-blocked system or one with correlators is tuned for the stream mode
 * only.  The timed sweeps are real moves: every walker set advances by
 * 2 * n_moves moves per shape tried (use it as burn-in).  Pass the number of moves per call that will be run: a launch
 * carries a fixed set-up cost (the first evaluation of every candidate) that
 * depends on the shape, so short timed sweeps can favour another shape than
 * long ones.  Blocks until the timing is done.
 */
vmc_status vmc_autotune(vmc_handle h, vmc_walkers* w, int32_t n_moves, int32_t* chosen, hipStream_t stream);
vmc_status vmc_batch_autotune(vmc_batch b, vmc_walkers* const* walkers, int32_t n_moves, int32_t* chosen,
                              hipStream_t stream);

/* Message of the last failed call on h (or of the last failed vmc_init /
 * handle-free call when h is NULL).  Valid until the next call on h. */
const char* vmc_last_error(vmc_handle h);

/*
 * Host-only table builder, for inspection without a GPU.  Builds the same
 * tables vmc_init uploads.  vmc_host_tables_get copies them out (any pointer
 * may be NULL):
 *   row_off [n_so*n_so + 1] int64: doubles of spin-orbital pair (i<j) are
 *           entries row_off[i*n_so+j] .. row_off[i*n_so+j+1]-1;
 *   dab     [E] int32 pairs (a, b) (2 per entry), dv [E] double v = <ab||ij>;
 *   s_off   [n_so + 1] int64, sa [S] int32, sS [S] double S_ia, sh [S] h_ia.
 */
typedef struct vmc_host_tables vmc_host_tables;
vmc_status vmc_host_tables_build(const vmc_system_desc* desc, const double* h1, const vmc_eri_list* eri, double eps,
                                 vmc_host_tables** out);
vmc_status vmc_host_tables_sizes(const vmc_host_tables* t, int64_t out[2]);
vmc_status vmc_host_tables_get(const vmc_host_tables* t, int64_t* row_off, int32_t* dab, double* dv, int64_t* s_off,
                               int32_t* sa, double* sS, double* sh);
void vmc_host_tables_free(vmc_host_tables* t);

#ifdef __cplusplus
}
#endif

#endif /* VMC_H */

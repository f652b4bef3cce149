/*
 * pmeqeq -- periodic Coulomb potentials, forces and energies (Ewald / smooth
 * particle-mesh Ewald) and charge equilibration (QEQ) on one AMD MI355X
 * (gfx950). C ABI.
 *
 * Method: Kaymak, Lubbers, Negre, Wall, Niklasson, "GPU-Accelerated
 * Charge-Equilibration for Shadow Molecular Dynamics in Python"
 * (arXiv:2503.21176).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Units: Angstrom, elementary charge e, eV. The Coulomb constant
 *   pq_coulomb_constant() = 14.3996454784 eV*A/e^2 multiplies every energy
 *   and potential.
 * - Array pointers are DEVICE pointers on the context's device (for example
 *   torch tensor data pointers), FP64, C-contiguous: positions and forces are
 *   n x 3 row-major (x, y, z per atom), per-atom vectors have n entries.
 *   Pointers documented as "host" are host memory.
 * - Calls are ordered on the context's HIP stream. A call returns after its
 *   work is enqueued unless it documents a host synchronisation; outputs are
 *   valid once the stream reaches that point. The caller owns every array it
 *   passes; the library never keeps a caller pointer after a call returns.
 * - Errors: every call returns a pq_status. Negative values are errors, in
 *   which case outputs are unspecified; pq_last_error() returns a message
 *   for the calling thread and pq_ctx_last_error(ctx) the context's last
 *   one. No C++ exception crosses this boundary.
 * - A context is not thread safe: one thread at a time per context.
 */
#ifndef PMEQEQ_H
#define PMEQEQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PQ_ABI_VERSION 5

typedef enum pq_status {
    PQ_OK = 0,
    PQ_WARN_NOT_CONVERGED = 1, /* solver stopped at max_it; outputs hold the last iterate */
    PQ_ERR_INVALID = -1,       /* bad argument (null pointer, size, parameter range) */
    PQ_ERR_BOX = -2,           /* box/cutoff/grid combination not supported */
    PQ_ERR_CAPACITY = -3,      /* caller buffer too small; required size reported */
    PQ_ERR_NOMEM = -4,         /* device allocation failed */
    PQ_ERR_HIP = -5,           /* HIP runtime error */
    PQ_ERR_TOO_LARGE = -6,     /* request larger than the server's memory budget,
                                  or a system beyond the list's index range */
    PQ_ERR_NAN = -7,           /* non-finite value in an input */
    PQ_ERR_STATE = -8,         /* call out of order (e.g. no system set) */
    PQ_ERR_TIMEOUT = -9        /* server poll timed out; the request is still pending */
} pq_status;

enum { PQ_METHOD_PME = 0, PQ_METHOD_EWALD = 1, PQ_METHOD_AUTO = 2 /* pq_choose_params only */ };

/* pq_params.flags bits.
 * PQ_FLAG_FP64: the per-atom bulk arithmetic (pair sum, spreading, FFT,
 *   convolution, gathering, direct-Ewald phases) runs in FP64 instead of the
 *   default FP32; every reduction is FP64 in both forms. The paper times
 *   everything but the neighbour search in double precision (Section
 *   "Performance"); this flag gives that form on the same kernels, for
 *   callers that need relative accuracy well below 1e-6. */
#define PQ_FLAG_FP64 1
/* PQ_FLAG_COMPENSATED (FP32 form): the real-space pair sums accumulate in
 *   FP32 blocks of 8 rounds that are folded into a running sum with an error
 *   term (TwoSum), and the lanes' partial sums are combined the same way, so
 *   the long per-atom sums lose no more than one FP32 rounding per block
 *   (compensated per-cell partial sums). Applies to the potential and
 *   force evaluations (pq_coulomb, the QEQ products); the two-charge force
 *   of pq_shadow_step and pq_qeq_vjp sums plainly. Ignored with
 *   PQ_FLAG_FP64. */
#define PQ_FLAG_COMPENSATED 2

/* Parameters of one periodic system. The names follow the paper's problem
 * statement for smooth PME (Algorithm "Smooth PME", input line: positions,
 * charges, box, Ewald parameter, grid dimensions, spline order) and the
 * regular Ewald sum (eqs. ewald_real, ewald_rec, ewald_self). */
typedef struct pq_params {
    double box[3];    /* box edges L_d in A, each > 0: the diagonal of the lattice  */
    double cutoff;    /* real-space cutoff rc in A, > 0; the erfc sum keeps |d| < rc  */
    double skin;      /* neighbour-list skin in A, >= 0 (list radius rc + skin)        */
    double alpha;     /* Ewald splitting parameter in 1/A, > 0                         */
    int32_t grid[3];  /* PME grid K_d: 2^a 3^b 5^c, 2*order <= K_d <= 1024             */
    int32_t order;    /* PME B-spline order p, 3 <= p <= 8                             */
    int32_t kmax[3];  /* direct Ewald: k = 2 pi n / L over |n_d| <= kmax_d, 0..64     */
    int32_t method;   /* PQ_METHOD_PME (grid, order used) or PQ_METHOD_EWALD (kmax)   */
    int32_t flags;    /* PQ_FLAG_FP64 | PQ_FLAG_COMPENSATED; other bits are rejected   */
    double tilt[3];   /* triclinic tilt factors (t_xy, t_xz, t_yz) in A; all 0 for an
                       * orthorhombic box. The lattice vectors are the rows of
                       *   a = (L0, 0, 0), b = (t_xy, L1, 0), c = (t_xz, t_yz, L2)
                       * (the general cell rotated so that a lies on x and b in the
                       * x-y plane), with |t_xy| <= L0/2, |t_xz| <= L0/2,
                       * |t_yz| <= L1/2 (any lattice has such a reduced basis; else
                       * PQ_ERR_BOX). Images are n0 a + n1 b + n2 c, wave vectors
                       * 2 pi H^-1 n, PME works on the fractional coordinates
                       * s = r H^-1 (the paper names triclinic cells for the Ewald
                       * sum, Section "Regular Ewald Summation"). With zero tilts
                       * every result is bit for bit that of the orthorhombic box.
                       * pq_md_run requires zero tilts (PQ_ERR_BOX). */
} pq_params;

/* Accuracy-driven parameters. The paper tunes the number of k-vectors of the
 * regular Ewald sum and the PME grid from a target Ewald accuracy delta with
 * the heuristics of OpenMM (Sections "Regular Ewald Summation", "Particle
 * Mesh Ewald Summation" and "Ewald Summation"; runs at delta = 5e-4, rc = 10).
 * The heuristics, as OpenMM documents them:
 *   alpha = sqrt(-ln(2 delta)) / rc
 *   Ewald: kmax_d = the smallest k >= max(1, ceil(L_d alpha / (pi sqrt 2)))
 *          (past the maximum of the estimate) with
 *          0.05 sqrt(L_d alpha) k exp(-(pi k / (L_d alpha))^2) <= delta
 *   PME:   K_d = the smallest 2^a 3^b 5^c >= max(ceil(2 alpha L_d / (3 delta^(1/5))), 2 p)
 * Inputs (host): box[3] > 0 (A), n >= 1 atoms, cutoff > 0 (A), 0 < delta <
 * 0.5, order p in 3..8, method PQ_METHOD_PME, PQ_METHOD_EWALD or
 * PQ_METHOD_AUTO. AUTO takes the direct Ewald sum below
 * pq_auto_pme_min_atoms() atoms (when its kmax fits 0..64) and PME from there
 * on: the crossover measured on MI355X for random ionic systems at rho 0.1/A^3,
 * delta 5e-4, rc 10 A, p 6. Writes *out completely (grid and kmax are both
 * filled; skin 0, flags 0). PQ_ERR_BOX if the chosen method's grid exceeds
 * 1024 or its kmax 64, PQ_ERR_INVALID for bad inputs. No device work. */
pq_status pq_choose_params(const double* box, int64_t n, double cutoff, double delta, int32_t order,
                           int32_t method, struct pq_params* out);
/* Atom count from which PQ_METHOD_AUTO chooses PME. */
int64_t pq_auto_pme_min_atoms(void);

/* Outcome of a Krylov solve (host struct filled by the library). */
typedef struct pq_solve_info {
    int32_t iterations;   /* matrix-vector products with the Coulomb operator      */
    int32_t restarts;     /* GMRES restarts performed                              */
    double rel_residual;  /* ||b - M z|| / ||b|| of the bordered system at exit    */
    double lambda;        /* Lagrange multiplier of the charge constraint          */
} pq_solve_info;

typedef struct pq_ctx pq_ctx;

/* ---- library ------------------------------------------------------------ */
int pq_abi_version(void);
/* e^2 / (4 pi eps0) in eV*A. */
double pq_coulomb_constant(void);
/* Message of the last failed call on this thread ("" if none). Valid until
 * the next call on the same thread. */
const char* pq_last_error(void);
/* Message of the last failed call on this context ("" if none, or for a NULL
 * context), whichever thread made it. Owned by the context; valid until the
 * next call on it or pq_destroy. */
const char* pq_ctx_last_error(const pq_ctx* ctx);

/* ---- context ------------------------------------------------------------ */
/* Device-memory allocator for a context's workspaces (the Python binding
 * passes torch's caching allocator). alloc(bytes, user_data) returns device
 * memory on the context's device, or NULL on failure (the call then returns
 * PQ_ERR_NOMEM); free(ptr, user_data) takes back a block that alloc
 * returned. Both are called on the thread that calls into the context, with
 * the context's device current. The library frees a block only after a
 * device-wide synchronisation, so no queued kernel still uses it. */
typedef struct pq_allocator {
    void* (*alloc)(size_t bytes, void* user_data);
    void (*free)(void* ptr, void* user_data);
    void* user_data;
} pq_allocator;

/* Creates a context on HIP device `device`; work is enqueued on `stream`
 * (a hipStream_t, NULL = the device's null stream). The context owns its
 * device workspaces (allocated on first use, grown on demand, freed by
 * pq_destroy), taken from `alloc` (copied; NULL, or NULL members:
 * hipMalloc / hipFree). */
pq_status pq_create(pq_ctx** out, int device, void* stream, const pq_allocator* alloc);
pq_status pq_set_stream(pq_ctx* ctx, void* stream);
pq_status pq_destroy(pq_ctx* ctx);

/* ---- system ------------------------------------------------------------- */
/* Sets the atoms' positions (device, n x 3 FP64, any real values: they are
 * wrapped into the box) and the parameters, and builds what depends on the
 * positions only (Section "Cell based Neighbor List"): the wrapped
 * coordinates, the cell (column) sort, the cluster-pair neighbour list
 * with radius rc + skin, and the PME B-spline stencils. Every periodic image
 * closer than rc is included, so boxes shorter than 2 rc are supported.
 * Host-synchronising (the list size is read back). Re-call when positions
 * move. 1 <= n; the clustered atom slots (n plus at most 7 padding slots per
 * x-y column) must stay below 2^24, else PQ_ERR_TOO_LARGE. A non-finite
 * coordinate is PQ_ERR_NAN. */
pq_status pq_set_system(pq_ctx* ctx, int64_t n, const double* pos, const pq_params* prm);

/* Moves the system's atoms to pos (device n x 3 FP64, the same atoms in the
 * same order) and keeps the neighbour list when every atom is within skin/2
 * of its position at the last full build: the list, built with radius
 * rc + skin, then still holds every pair closer than rc (the paper's skin
 * rule for re-neighbouring, Section "Performance"). The cluster-pair search
 * is skipped; the atoms' list positions, the pair decisions (the canonical
 * FP64 predicate at rc on the current positions, with image vectors that
 * follow atoms across the cell faces) and the PME stencils are redone.
 * Otherwise (an atom moved further, skin == 0, a triclinic cell) it is
 * pq_set_system(pos) with the current parameters. *rebuilt (host, may be
 * NULL) = 1 if a full build ran. Host-synchronising (the largest
 * displacement is read back). */
pq_status pq_update_positions(pq_ctx* ctx, const double* pos, int32_t* rebuilt);

/* Number of neighbour pairs (i, j, n) with |w_j - w_i + n L| < rc + skin,
 * each unordered pair once (i < j, or i == j with the image vector n
 * lexicographically positive), evaluated with the canonical FP64 predicate
 * d.d < (rc+skin)^2 on the wrapped positions. Host-synchronising.
 * After pq_update_positions kept the list, the pairs closer than rc (the
 * kept list covers those), with the image vectors of the current wrapped
 * positions. `pairs` (device int32, 5 x cap, row-major rows i, j, n0, n1,
 * n2, in no particular order) may be NULL to query the count only; if cap is too small
 * the call returns PQ_ERR_CAPACITY with *n_pairs (host) set to the count. */
pq_status pq_neighbor_pairs(pq_ctx* ctx, int64_t cap, int32_t* pairs, int64_t* n_pairs);

/* The same neighbour set in the ELLPACK form of Section "Cell based Neighbor
 * List" (an n x K matrix, K the largest neighbour count). Row i lists every
 * neighbour (j, n) of atom i: both directions of each pair of
 * pq_neighbor_pairs ((i, j, n) gives (j, n) in row i and (i, -n) in row j; an
 * atom's own images appear as (i, n) and (i, -n)), in ascending order of
 * (j, n0, n1, n2), then padding. Outputs (device, each may be NULL):
 *   nbr[n*K]    int32 row-major neighbour indices, -1 in the padding;
 *   img[n*K*3]  int32 image vectors of the entries, 0 in the padding;
 *   count[n]    int32 neighbours per row.
 * *k_max (host, required) = the largest row count. With nbr or img given,
 * K < *k_max returns PQ_ERR_CAPACITY (nothing written to nbr or img, count
 * written), and *k_max > PQ_ELL_MAX_K returns PQ_ERR_TOO_LARGE. Uses a
 * temporary device buffer of n*K*8 bytes. Host-synchronising. */
#define PQ_ELL_MAX_K 8192
pq_status pq_neighbor_ell(pq_ctx* ctx, int32_t K, int32_t* nbr, int32_t* img, int32_t* count, int32_t* k_max);

/* ---- Coulomb evaluation ------------------------------------------------- */
/* Periodic Coulomb potential, force and energy of the charge vector q
 * (device, n FP64; need not be neutral):
 *   phi_i = dE_Coul/dq_i = KE [ sum_{(j,n) != (i,0), |d| < rc} q_j erfc(a|d|)/|d|
 *                               + reciprocal(i) - 2 a/sqrt(pi) q_i - pi Q/(V a^2) ]
 *   F_i   = -dE_Coul/dr_i,   E_Coul = 1/2 sum_i q_i phi_i,
 * the Ewald split of the paper's eqs. ewald_general, ewald_real, ewald_rec and
 * ewald_self, with the reciprocal part by smooth PME (Algorithm "Smooth PME",
 * steps 1-5) or by the direct k-sum, and a neutralising background term
 * (zero for neutral q). Outputs (device, FP64, each may be NULL):
 *   phi[n], force[n*3], energy[4] = {E_Coul, E_real, E_rec, E_self+background}.
 * Bulk arithmetic is FP32; energies and charge sums are reduced in FP64.
 * Charges are not checked: a non-finite charge makes the outputs
 * non-finite. */
pq_status pq_coulomb(pq_ctx* ctx, const double* q, double* phi, double* force, double* energy);

/* ---- Coulomb evaluation without device allocation ------------------------ */
/* For callers that cannot allocate device memory during the call: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same evaluation and outputs as pq_coulomb (bitwise the same values); the
 * FP64 reduction partials and the evaluation's device scalars live in a
 * static device array of PQ_NOALLOC_SCRATCH_BYTES per device (held until the
 * process ends) instead of context buffers, and the pair kernel runs on the
 * context's stream. The call allocates and frees nothing: pq_set_system must
 * have been called on the context (it sizes the per-atom buffers), and
 * phase timing must be off (PQ_ERR_STATE otherwise). PQ_ERR_TOO_LARGE, with
 * nothing launched, if the PME grid needs more than the scratch holds:
 * (grid[0]/2 + 1) * grid[1] + 16 partial sums must fit in
 * PQ_NOALLOC_SCRATCH_BYTES/8 - 592 doubles (grid[0] = grid[1] <= 509).
 * Every call on one device shares that device's scratch array: calls that
 * overlap on the same device (two contexts, two streams, two threads) race
 * and must be ordered by the caller. */
#define PQ_NOALLOC_SCRATCH_BYTES (1u << 20)
pq_status pq_coulomb_noalloc(pq_ctx* ctx, const double* q, double* phi, double* force, double* energy);

/* ---- phase timing ---------------------------------------------------------- */
/* Phases of one Coulomb evaluation, timed with HIP events recorded on the
 * context's stream around each phase's kernels (the time the device spends
 * from the phase's first kernel start to its last kernel end). */
enum {
    PQ_PHASE_STAGE = 0,    /* charge staging and FP64 charge sum              */
    PQ_PHASE_PAIR = 1,     /* real-space pair kernel                          */
    PQ_PHASE_SPREAD = 2,   /* grid clear + B-spline spreading (PME)           */
    PQ_PHASE_FFT = 3,      /* forward FFT, convolution, inverse FFT (PME)     */
    PQ_PHASE_GATHER = 4,   /* gather (PME) or structure factors + k-sum (Ewald) */
    PQ_PHASE_COMBINE = 5,  /* self/background terms, outputs, FP64 energies   */
    PQ_PHASE_TOTAL = 6,    /* whole evaluation                                */
    PQ_NPHASE = 7
};
/* Event timing of pq_coulomb and of the evaluations inside the solvers:
 * on = 0 off; 1 on (the real-space phase overlaps the reciprocal phases on a
 * second stream as usual, so their intervals overlap); 2 on with the phases
 * serialised on the context's stream, so each phase is timed alone. Adds two
 * events per phase per evaluation. */
pq_status pq_set_timing(pq_ctx* ctx, int on);
/* Host-synchronising. Writes to ms[0..PQ_NPHASE) (host) the milliseconds
 * summed over the evaluations timed since the last call, and to *count the
 * number of those evaluations; then resets both. */
pq_status pq_timings(pq_ctx* ctx, double* ms, int64_t* count);

/* ---- charge equilibration ----------------------------------------------- */
/* Krylov method of a context's QEQ solves (pq_qeq_solve, pq_qeq_vjp and the
 * regular mode of pq_md_run); the paper solves the system with GMRES, CG "or
 * related approaches" (Section "Regular Born-Oppenheimer MD for a Charge
 * Equilibration Model"), and C is indefinite when pairs closer than
 * KE/sqrt(u_i u_j) exist, which rules out CG:
 *   PQ_SOLVER_GMRES   restarted GMRES(restart), Jacobi diag(u, 1) on the right
 *                     (the default);
 *   PQ_SOLVER_MINRES  preconditioned MINRES on the symmetric bordered matrix
 *                     with the SPD preconditioner diag(u, 1) (Paige and
 *                     Saunders): short recurrences, O(n) memory, no restart
 *                     length.
 * vjp_restart (1..PQ_MAX_RESTART) is the GMRES restart length of the adjoint
 * solve in pq_qeq_vjp (default 50). */
enum { PQ_SOLVER_GMRES = 0, PQ_SOLVER_MINRES = 1 };
#define PQ_MAX_RESTART 4096
pq_status pq_set_solver(pq_ctx* ctx, int32_t solver, int32_t vjp_restart);

/* Regular QEQ (Section "Regular Born-Oppenheimer MD for a Charge
 * Equilibration Model"): minimise E(q) = sum q chi + 1/2 sum u q^2 + E_Coul(q)
 * subject to sum q = q_tot, i.e. solve the bordered system of eq. linear_qeq
 *   [[C, 1], [1^T, 0]] [q; lambda] = [-chi; q_tot],  C v = u o v + phi[v]
 * matrix-free (the paper's Cv identity) by the context's Krylov method
 * (pq_set_solver): restarted GMRES(restart) (1 <= restart <= PQ_MAX_RESTART;
 * restart >= max_it is full GMRES) with the Jacobi preconditioner diag(u, 1)
 * applied on the right, or preconditioned MINRES (restart ignored); FP64
 * Krylov vectors and FP64 orthogonalisation, each product one FP32-bulk
 * Coulomb evaluation. Stops when the true relative residual
 * ||b - M z||/||b|| <= tol or after max_it products (PQ_WARN_NOT_CONVERGED,
 * last iterate returned; info->rel_residual holds its true residual).
 *   chi, eta (= u): device n FP64; q0: device n FP64 start vector or NULL (0);
 *   q: device n FP64 output; force: device n*3 FP64 output F = -dE/dR at the
 *   solution, or NULL; energy: device FP64[1] output E(q), or NULL;
 *   info: host, may be NULL. Host-synchronising (convergence checks).
 * Each solver step (operator product, then orthogonalisation and Givens
 * update, or the MINRES recurrences) is one launch of a HIP graph that the
 * context builds at its first solve of a system and reuses across restarts
 * and calls; the host reads the residual estimate of step j - 1 while step j
 * runs, so a solve may execute one product beyond the step it converges at
 * (counted in info->iterations). */
pq_status pq_qeq_solve(pq_ctx* ctx, const double* chi, const double* eta, double q_tot,
                       double tol, int max_it, int restart, const double* q0,
                       double* q, double* force, double* energy, pq_solve_info* info);

/* One shadow-MD charge step (Section "Shadow Born-Oppenheimer MD"):
 *   v = phi[n_vec]; q[n] from the quasi-diagonal system of eq. diag_linear_qeq
 *   (lambda in closed form, FP64 reductions); the shadow force
 *   F = -d/dR of the shadow energy (eq. qeq_energy) at fixed n and q[n],
 *   computed as F[q] - F[q - n]; and the n_krylov-step GMRES iterate x from
 *   x0 = 0 for J x = -(q[n] - n) (eq. Jnddot with omega^2 = 1),
 *   J = -I - P D^-1 A, P = I - D^-1 1 1^T / (1^T D^-1 1), D = diag(u).
 * Fixed work: 1 potential + 2 force evaluations + n_krylov products (each
 * Krylov step one graph launch, as in pq_qeq_solve); no host
 * synchronisation. Outputs (device FP64): q_n[n], force[n*3] (may be NULL),
 * nddot[n] (may be NULL), energy[2] = {shadow energy, lambda} (may be NULL). */
pq_status pq_shadow_step(pq_ctx* ctx, const double* chi, const double* eta, double q_tot,
                         const double* n_vec, int n_krylov,
                         double* q_n, double* force, double* nddot, double* energy);

/* Vector-Jacobian product through the regular QEQ solution q*(R, chi, u)
 * (training through the solve, Section "Validation and Performance"):
 * adjoint solve [[C,1],[1^T,0]] [a; mu] = [gbar; 0] (the context's Krylov
 * method, GMRES with the restart length set by pq_set_solver, to tol),
 * then dL/dchi = -a, dL/du_i = -a_i q*_i, dL/dR = F[a + q*] - F[a] - F[q*].
 * With gbar == NULL the upstream is the QEQ energy itself and the envelope
 * theorem gives dE/dR = -F[q*], dE/dchi = q*, dE/du = q*^2/2 (no solve).
 * q_star: device n FP64 (the solution of pq_qeq_solve for this system).
 * Outputs (device FP64, each may be NULL): d_pos[n*3], d_chi[n], d_eta[n]. */
pq_status pq_qeq_vjp(pq_ctx* ctx, const double* chi, const double* eta, const double* q_star,
                     const double* gbar, double tol, int max_it,
                     double* d_pos, double* d_chi, double* d_eta);

/* ---- autotuning ------------------------------------------------------------ */
/* Launch shape of the real-space pair kernel: 0 runs one wavefront per
 * i-cluster (every cluster in flight at once); k > 0 runs k workgroups per CU
 * that stride over the clusters, leaving LDS and wave slots of every CU to the
 * reciprocal-space kernels that run concurrently on the context's other
 * stream. Every shape gives bitwise-identical results. */
typedef struct pq_tune_result {
    int32_t pair_wg_per_cu;   /* chosen pair-kernel shape (0 or workgroups per CU)     */
    int32_t candidates;       /* configurations timed                                  */
    double ms;                /* mean phi+F evaluation time of the choice, ms          */
    double ms_default;        /* the same for shape 0 and the default FFT tiles        */
    int32_t fft_lds_bytes;    /* LDS bytes per FFT ping-pong buffer (0: default 18432); */
                              /* smaller tiles let FFT workgroups run beside the pair  */
                              /* kernel; the results do not depend on it               */
    int32_t pair_fork;        /* PME: where the pair kernel's stream forks: 0 before   */
                              /* the reciprocal chain, 1 after the first spreading     */
                              /* pass, 2 after spreading; the results do not depend    */
                              /* on it                                                 */
} pq_tune_result;

/* Times the pair-kernel shapes 0, 1, 2, 3, 4, 6, 8 jointly with FFT buffer
 * sizes of 18432, 9216 and 4608 bytes and (PME) the fork points 0, 1, 2 on
 * `reps` (1..1000) potential + force evaluations each, after one warm-up, of
 * the current system with charges q (device, n); the four fastest are timed
 * again twice, interleaved, on 2 x reps evaluations each, and the fastest mean
 * is kept for this context (also across later pq_set_system calls; out->ms is
 * that mean). Phase timing must be off. Host-synchronising; out may be NULL.
 * If tuning fails, the context keeps the choice it had before the call. */
pq_status pq_autotune(pq_ctx* ctx, const double* q, int32_t reps, pq_tune_result* out);
/* Applies a stored choice (pair_wg_per_cu in 0..64; fft_lds_bytes 0 or
 * 1024..65536; pair_fork 0..2). */
pq_status pq_set_tuning(pq_ctx* ctx, const pq_tune_result* t);

/* ---- shadow MD driver ----------------------------------------------------- */
/* Shadow Born-Oppenheimer (XL-BOMD) molecular dynamics on the context's
 * system (Section "Shadow Born-Oppenheimer MD for a Charge Equilibration
 * Model"): the atoms move on the shadow potential with the force at fixed n
 * (velocity Verlet); the extended charges follow n'' = -omega^2 K (q[n] - n),
 * whose right-hand side each step approximates with n_krylov GMRES steps on
 * J x = -(q[n] - n), integrated as
 *   n(t+dt) = 2 n(t) - n(t-dt) + kappa x(t) + alpha sum_k c_k n(t - k dt)
 * (kappa = dt^2 omega^2). dissipation = 5 takes the weak-dissipation scheme
 * of extended-Lagrangian BOMD with K = 5 (kappa 1.82, alpha 0.018,
 * c = -6, 14, -8, -3, 4, -1); dissipation = 0 uses alpha = 0 and the given
 * kappa. After each position update the system is moved with
 * pq_update_positions: the neighbour list is kept while every atom stays
 * within skin/2 of its position at the last full build (the context's
 * pq_params.skin; skin 0 rebuilds every step) and rebuilt otherwise (the
 * paper's skin rule, Section "Performance"). V_short, the paper's trained short-range model, is not part of
 * this library: a repulsive pair term rep_a exp(-r/rep_rho) over every pair
 * and image closer than the cutoff stands in for it (rep_a = 0: none; brute
 * force over all pairs, FP64, meant for test systems of a few thousand atoms).
 * mode PQ_MD_REGULAR runs regular Born-Oppenheimer MD instead (Section
 * "Regular Born-Oppenheimer MD for a Charge Equilibration Model"): every step
 * solves the QEQ system with pq_qeq_solve to relative residual tol (max_it
 * products, GMRES(restart)), started from the previous step's charges, and
 * moves the atoms with the force at those charges; n_hist[0] holds the start
 * charges on entry and the last charges on return.
 * Units: A, fs, amu, eV. */
enum { PQ_MD_SHADOW = 0, PQ_MD_REGULAR = 1 };
typedef struct pq_md_cfg {
    double dt_fs;          /* time step in fs, > 0                                  */
    int32_t n_krylov;      /* Krylov steps for n'' per MD step, 1..512               */
    int32_t dissipation;   /* 0 or 5 (see above)                                    */
    double kappa;          /* dt^2 omega^2 when dissipation = 0                      */
    double rep_a, rep_rho; /* V_short stand-in: A (eV) >= 0, rho (A) > 0 when A > 0  */
    int32_t mode;          /* PQ_MD_SHADOW or PQ_MD_REGULAR                          */
    int32_t max_it;        /* regular mode: products per solve, >= 1                 */
    int32_t restart;       /* regular mode: GMRES restart length, >= 1               */
    int32_t reserved;
    double tol;            /* regular mode: relative residual of each solve, > 0     */
} pq_md_cfg;

/* Runs `steps` steps from the state in pos, vel (device n x 3 FP64, updated
 * in place; the context must already hold a system of n atoms and the
 * parameters to run with, from pq_set_system) and n_hist (device,
 * pq_md_history() vectors of n, newest first: n(t), n(t - dt), ...; updated
 * in place). pos_ref (device n x 3 FP64, or NULL): the positions of the last
 * full neighbour build; on entry the list is built there and moved to pos,
 * on return it holds the positions of the run's last full build. NULL: the
 * list is built at pos. (pos, vel, n_hist, pos_ref) is the whole state of
 * a run: a run continued from a saved copy of it, in a fresh context with the
 * same parameters, repeats the uninterrupted run bit for bit (for a fresh
 * start pass a copy of pos as pos_ref). mass (amu), chi, eta (= u): device n
 * FP64. energies: host (steps + 1) x 6 FP64 or NULL, row t = {kinetic,
 * potential (shadow energy E(R, q[n], n), or the QEQ energy E(R, q) in
 * regular mode), V_short, total, Coulomb evaluations of that step's force
 * evaluation, 1 if the neighbour list was rebuilt for it (else 0)} at step t
 * (row 0: the initial state). Host-synchronising. */
pq_status pq_md_run(pq_ctx* ctx, double* pos, double* vel, const double* mass, const double* chi,
                    const double* eta, double q_tot, double* n_hist, double* pos_ref, int32_t steps,
                    const pq_md_cfg* cfg, double* energies);
/* Number of n vectors pq_md_run keeps for a dissipation setting (2 or 6). */
int32_t pq_md_history(int32_t dissipation);

/* ---- continuous-batching QEQ server -------------------------------------- */
/* A server owns `slots` contexts on one device, each with its own HIP stream
 * and worker thread, and a scheduler thread. Submitted requests wait in FIFO
 * order and are admitted when a slot is free and their estimated
 * device-memory footprint fits the remaining budget; each admitted request
 * runs its neighbour build and GMRES solve on its slot's stream, so the
 * kernels of all admitted requests overlap on the device and new requests
 * start as soon as earlier ones release a slot and memory. Slots launch their
 * kernels directly (no Arnoldi-step graphs). */
typedef struct pq_server pq_server;

typedef struct pq_server_cfg {
    int32_t device;
    int32_t slots;            /* concurrent requests on the device, 1..64       */
    double hbm_budget_bytes;  /* admission limit on summed request footprints   */
} pq_server_cfg;

/* A request: all pointers are HOST memory, copied at submit. */
typedef struct pq_request {
    int64_t n;
    const double* pos;        /* n x 3 */
    const double* chi;        /* n     */
    const double* eta;        /* n     */
    const double* q0;         /* n or NULL */
    double q_tot;
    double tol;
    int32_t max_it;
    int32_t restart;
    int32_t solver;           /* PQ_SOLVER_GMRES or PQ_SOLVER_MINRES */
    int32_t reserved;         /* 0 */
    pq_params params;
} pq_request;

/* Result: `q` is a HOST buffer of n doubles provided by the caller of poll. */
typedef struct pq_result {
    double* q;
    double energy;
    pq_solve_info info;
    int32_t status;           /* pq_status of the solve */
    double t_submit_s, t_start_s, t_done_s;   /* server clock, seconds */
    char message[256];        /* for an error status: what failed (NUL-terminated) */
} pq_result;

pq_status pq_server_create(pq_server** out, const pq_server_cfg* cfg);
/* Copies the request; returns PQ_ERR_TOO_LARGE if its footprint exceeds
 * the whole budget. *ticket identifies it for poll. Thread safe. */
pq_status pq_server_submit(pq_server* s, const pq_request* req, uint64_t* ticket);
/* Waits up to timeout_us (< 0: forever) for the request; on completion copies
 * the result out (res->q must hold n doubles) and forgets the ticket. Returns
 * PQ_ERR_TIMEOUT if still pending. Thread safe. */
pq_status pq_server_poll(pq_server* s, uint64_t ticket, pq_result* res, int64_t timeout_us);
/* Runs the requests already submitted to completion, stops the scheduler and
 * the slots and frees the server (results not polled are dropped). No other
 * call on the same server may run concurrently with it or follow it. */
pq_status pq_server_destroy(pq_server* s);
/* The footprint in bytes that admission charges for a request of n atoms with
 * these parameters and GMRES restart length (an estimate of the device memory
 * it holds while running: neighbour lists, per-atom arrays, PME grids, Krylov
 * basis). -1 for invalid arguments. Host only, no device call. */
double pq_request_footprint(int64_t n, const pq_params* params, int32_t restart);

#ifdef __cplusplus
}
#endif
#endif /* PMEQEQ_H */

/*
 * fmm355.h -- C ABI of the MI355X (gfx950) symmetric FMM gravity solver and
 * hierarchical-Hamiltonian-splitting (HHS) integrator.
 *
 * The method is that of Q. Zhu, "A momentum conserving N-body scheme with
 * individual timesteps" (arXiv:1712.10116):
 *   - a fast multipole (FMM) gravity solve on an oct-tree whose dual tree walk
 *     opens BOTH cells of a pair that fails the well-separation test, so that
 *     the cell-cell (M2L) and leaf-leaf (P2P) interaction lists are symmetric
 *     and every interaction acts on both sides (Sec. 2.1, Eq. (1)-(2);
 *     Sec. 2.3, Algorithm 4);
 *   - the HOLD/HHS integrator that splits particles into slow and fast systems
 *     on power-of-two timestep rungs, with kickS2F forces computed by masking
 *     the masses of the fast system (Sec. 2.2, Algorithms 1-3; Sec. 2.3);
 *   - around them: the individual-timestep integrator the paper compares
 *     against (Sec. 2.3), the total-acceleration timestep bound (Eq. (9)),
 *     the comoving drift and kick factors and the HHS in comoving form
 *     (Sec. 3.5, Eqs. (10)-(11)), and the force gradient that a fourth-order
 *     integrator needs (Sec. 4.1).
 *
 * Conventions for every call
 *   - Units: G = 1.  Outputs are accelerations per unit mass,
 *     a_i = -grad_i Phi_i, and potentials Phi_i = sum_{j != i} m_j psi(r_ij),
 *     psi < 0 (Wendland C2 softening of Eq. (8), or Plummer softening).
 *   - Particle arrays are structure-of-arrays in DEVICE memory: a position
 *     array of n_total particles is x[0..n_total) followed by y and z (3 x
 *     n_total doubles); masses are n_total doubles.  The caller owns every
 *     particle, index and output buffer; the library owns its workspace.
 *   - "active" lists n_active distinct indices into [0, n_total) (int32, device
 *     memory); NULL means all n_total particles in order (n_active = n_total).
 *     n_active = 0 is always valid and does nothing.  Outputs are written
 *     in active-list order (output slot s belongs to particle active[s]).
 *   - Every call is ordered on the stream given to fmm_create.  Argument
 *     errors are returned synchronously without touching the GPU.  fmm_build
 *     waits for its own work (it reads back list sizes); fmm_evaluate and
 *     fmm_forces return once their kernels are queued.
 *   - No call aborts the process.  On any status other than FMM_OK,
 *     fmm_last_error() describes the failure.
 *   - A context is not thread safe; use one context per host thread.
 */
#ifndef FMM355_H
#define FMM355_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FMM_OK = 0,
    FMM_EINVAL = 1,      /* bad argument (sizes, parameters, NULL pointers)      */
    FMM_ENOMEM = 2,      /* device allocation failed                              */
    FMM_EDEVICE = 3,     /* a HIP runtime call failed                             */
    FMM_ENONFINITE = 4,  /* an input position was NaN or infinite                 */
    FMM_ESTALE = 5,      /* fmm_evaluate without a tree built for these particles */
    FMM_EOVERFLOW = 6    /* a list or tree exceeded its workspace after regrowth  */
} fmm_status;

typedef enum {
    FMM_KERNEL_WENDLAND_C2 = 0, /* Eq. (8): Wendland C2 inside eps, -1/r outside   */
    FMM_KERNEL_PLUMMER = 1      /* psi = -(r^2 + eps^2)^(-1/2)                     */
} fmm_kernel;

typedef enum {
    FMM_PREC_FP64 = 0,  /* every step in IEEE double                                */
    FMM_PREC_MIXED = 1  /* P2P, M2L and the expansions in FP32 on cell-local, size-
                           scaled quantities; positions, centres, accumulation of
                           the near field and the outputs in FP64                  */
} fmm_precision;

/* Solver parameters fixed for the life of a context. */
typedef struct {
    int p_max;          /* largest expansion order a call may ask for (1..8)       */
    int leaf_size;      /* n_crit: a cell splits while it holds more particles (>=1) */
    int kernel;         /* fmm_kernel                                              */
    int precision;      /* fmm_precision                                           */
} fmm_params;

typedef struct fmm_ctx fmm_ctx;

/* Create a solver context on the current HIP device for up to max_n active
 * particles per call.  stream: a hipStream_t (NULL = the null stream).
 * Allocates the whole workspace; later calls allocate only if the cells or an
 * interaction list outgrow their estimate (that buffer is then regrown, at
 * least doubling, and the build repeated). */
fmm_status fmm_create(const fmm_params *prm, int64_t max_n, void *stream, fmm_ctx **out);
fmm_status fmm_destroy(fmm_ctx *ctx);
const char *fmm_last_error(const fmm_ctx *ctx);

/* Geometry-only part of the solve (independent of masses): root box, 63-bit
 * Morton keys (21 bits per axis), stable key sort, top-down oct-tree split
 * while a cell holds more than leaf_size particles (to depth 21), geometric
 * cell centres, and the symmetric dual walk producing the M2L and P2P lists.
 * Well-separation (Eq. (1) with R = cell half side, plus the softening rule of
 * Sec. 2.3): |zA-zB|^2 theta^2 > (hA+hB)^2 and
 * |zA-zB|^2 > (eps + sqrt(3)(hA+hB))^2.
 * pos: device, 3 x n_total doubles.  active: device int32[n_active] or NULL.
 * Requires 0 <= n_active <= max_n, 0 < theta, eps >= 0.  Blocks until the tree
 * and lists are complete.  The tree stays valid for fmm_evaluate until the
 * next fmm_build/fmm_forces on this context. */
fmm_status fmm_build(fmm_ctx *ctx, const double *pos, int64_t n_total, const int32_t *active,
                     int64_t n_active, double eps, double theta);

/* Mass-dependent part on the tree of the last fmm_build: P2M, M2M (upward),
 * M2L over the symmetric cell-pair list, P2P over the symmetric leaf-pair list,
 * L2L (downward), L2P.  pos/active/n_active must be those of the build (else
 * FMM_ESTALE).  mass: device, n_total doubles (zeros allowed: masked sources).
 * acc: device, 3 x n_active doubles (SoA); pot: device, n_active doubles.
 * 1 <= p <= p_max.  Asynchronous on the context's stream. */
fmm_status fmm_evaluate(fmm_ctx *ctx, const double *pos, const double *mass, int64_t n_total,
                        const int32_t *active, int64_t n_active, int p, double *acc,
                        double *pot);

/* fmm_build followed by fmm_evaluate: acceleration and potential of every
 * active particle due to all active masses (the Poisson solve called by each
 * kick of Algorithm 3).  The masses being known when the tree is built, the
 * mass gather, P2M and M2M run on the context's second stream beside the
 * walk; the results equal fmm_build + fmm_evaluate bit for bit. */
fmm_status fmm_forces(fmm_ctx *ctx, const double *pos, const double *mass, int64_t n_total,
                      const int32_t *active, int64_t n_active, double eps, double theta,
                      int p, double *acc, double *pot);

/* fmm_forces plus the force gradient d a_i / d x_i of every active particle
 * (the tidal tensor that the fourth-order integrator of Sec. 4.1 needs from
 * the FMM), from the same tree, lists and local expansions: minus the Hessian
 * of the leaf's local expansion (exact derivative of the truncated expansion;
 * zero for p = 1), plus for every particle j of the P2P partners the
 * derivative of m_j g(r) d, d = x_j - x_i, with respect to x_i,
 * -m_j (g I + (dg/dr)/r d d^T), in the context's precision (pair terms on
 * FP64 differences, summed into FP64 per source leaf).
 * grad: device, 6 x n_active doubles (SoA rows xx, yy, zz, xy, xz, yz), in
 * active order.  The first call allocates 6 x max_n doubles in the context
 * (the near part, staged in Morton order).  Errors as fmm_forces, and
 * FMM_EINVAL for a NULL grad, FMM_ENOMEM if that staging does not fit. */
fmm_status fmm_forces_grad(fmm_ctx *ctx, const double *pos, const double *mass, int64_t n_total,
                           const int32_t *active, int64_t n_active, double eps, double theta,
                           int p, double *acc, double *pot, double *grad);

/* The field of vector sources on the tree of the last fmm_build /
 * fmm_forces / fmm_forces_grad (one system; same pos, active, n_total and
 * n_active, else FMM_ESTALE): every active particle j carries the vector
 * m_j v_j, and
 *   u_i   = sum_{j != i} m_j H(x_i - x_j) v_j,   H = grad grad psi
 *           (the pair Hessian g I + (dg/dr)/r d d^T of the softened kernel),
 *   phi_i = sum_{j != i} m_j v_j . grad psi(x_i - x_j).
 * u_i is the derivative of a_i along a displacement of every other particle j
 * by v_j, sum_j (d a_i / d x_j) v_j; with v = a it is the cross term of the
 * force-gradient kick of the fourth-order integrator of Sec. 4.1.  Computed
 * through the same expansions as the forces: each source's moments are the
 * derivative of its mass moments along v_j (total degree <= p), the same
 * M2M, M2L and L2L, u = +grad of the local expansion at L2P, and the P2P
 * partners summed directly (context precision, as fmm_forces_grad).
 * vec, u: device SoA 3 x n_active; phi: device n_active; all in active
 * order.  The first call allocates 3 x max_n doubles of scratch in the
 * context.  FMM_EINVAL for NULL arrays, a batched tree or p outside 1..p_max;
 * asynchronous on the context's stream. */
fmm_status fmm_evaluate_dipole(fmm_ctx *ctx, const double *pos, const double *mass,
                               int64_t n_total, const int32_t *active, int64_t n_active, int p,
                               const double *vec, double *u, double *phi);

/* ---------------------------------------------------------------------------
 * Forward fourth-order integrator (Sec. 4.1: Chin & Chen 2005, algorithm 4A)
 * with one shared timestep h:  v += h/6 a;  x += h/2 v;  v += 2h/3 a~;
 * x += h/2 v;  v += h/6 a, where the middle kick uses the modified
 * acceleration a~_i = a_i + (h^2/24) sum_j (d a_i / d x_j) a_j
 * = a_i + (h^2/24) (T_i a_i + u_i), T_i the force gradient of fmm_forces_grad
 * and u_i the field of the vector sources m_j a_j (fmm_evaluate_dipole).
 * Per step: two trees, three evaluations (forces with the gradient, the
 * vector-source pass, forces at the end, whose acceleration opens the next
 * step).  Kicks and drifts FP64.
 * ------------------------------------------------------------------------- */
typedef struct {
    double *pos;        /* device, 3 x n SoA (updated in place)                */
    double *vel;        /* device, 3 x n SoA (updated in place)                */
    const double *mass; /* device, n                                           */
    double *acc;        /* device, 3 x n: acceleration at pos (set by chin_init
                           and by every step)                                  */
    double *work;       /* device scratch of chin_work_bytes(n) bytes, owned by
                           the caller, not read between calls                  */
    int64_t n;          /* 1 .. max_n of the context                           */
    double t;           /* advanced by h per step                              */
} chin_state;

/* Bytes of the work array for n particles (13 n doubles); -1 for n < 1. */
int64_t chin_work_bytes(int64_t n);
/* acc = acceleration at pos (one fmm_forces); needed once before chin_step. */
fmm_status chin_init(fmm_ctx *ctx, chin_state *st, double eps, double theta, int p);
/* One step of length h (h != 0 and finite: a negative h steps backwards, the
 * scheme being time symmetric).  stats (host, may be NULL): [0] evaluations
 * (3), [1] particles summed over them, [2] tree builds (2).  FMM_EINVAL for a
 * bad state or h; errors of the solves are passed on. */
fmm_status chin_step(fmm_ctx *ctx, chin_state *st, double eps, double theta, int p, double h,
                     int64_t stats[3]);

/* ---------------------------------------------------------------------------
 * Comoving integration factors (Sec. 3.5, Eqs. 10-11): the drift operator
 * moves comoving positions by p/m times the integral of dt/a^2 over the step,
 * the kick operator changes the canonical momenta by the force times the
 * integral of dt/a; both are kept in a lookup table over the scale factor a.
 * Host-side only (no device memory, no GPU work).
 * ------------------------------------------------------------------------- */
typedef struct {
    double omega_m;  /* matter density parameter (>= 0)                        */
    double omega_l;  /* cosmological constant; curvature 1 - omega_m - omega_l */
    double h0;       /* Hubble constant in the integrator's time unit (> 0)     */
    double a_min, a_max; /* table range of the scale factor, 0 < a_min < a_max */
    int n;           /* grid points, uniform in ln a (2 .. 2^24)                */
} fmm_cosmo_params;
typedef struct fmm_cosmo fmm_cosmo;

/* Builds the table: integrals of dt/a^2 and dt/a over each grid interval,
 * with dt = d(ln a) / H(a), H = h0 sqrt(omega_m a^-3 + (1 - omega_m - omega_l) a^-2
 * + omega_l), each grid interval by 8-point Gauss-Legendre.  FMM_EINVAL for
 * bad parameters or H^2 <= 0 inside the range; FMM_ENOMEM. */
fmm_status fmm_cosmo_create(const fmm_cosmo_params *prm, fmm_cosmo **out);
/* drift = integral of dt/a^2 and kick = integral of dt/a from a0 to a1 (both
 * inside the table's range; a1 < a0 gives negative factors): the intervals
 * between them from the table plus the two partial intervals by the same
 * rule.  FMM_EINVAL for a NULL argument or a scale factor outside the range. */
fmm_status fmm_cosmo_factors(const fmm_cosmo *tab, double a0, double a1, double *drift,
                             double *kick);
fmm_status fmm_cosmo_destroy(fmm_cosmo *tab);

/* ---------------------------------------------------------------------------
 * Batched solves: several independent particle systems in one set of launches
 * ------------------------------------------------------------------------- */

/* One independent system of a batch.  pos/active/n_total/n_active as for
 * fmm_build; mass, acc and pot as for fmm_evaluate (ignored by the build).
 * Each system gets its own root box, Morton keys and root cell; the walk
 * starts every root only against itself, so no cell of one system ever meets
 * a cell of another, and each system's tree, lists and results are exactly
 * those of a solve of that system alone. */
typedef struct {
    const double *pos;      /* device, 3 x n_total doubles (SoA)              */
    int64_t n_total;
    const int32_t *active;  /* device int32[n_active], or NULL = all n_total    */
    int64_t n_active;
    const double *mass;     /* device, n_total doubles; NULL in an evaluation:
                               the system is skipped, acc/pot left untouched   */
    double *acc;            /* device, 3 x n_active doubles (out)              */
    double *pot;            /* device, n_active doubles (out)                  */
    const uint8_t *sinks;   /* device uint8[n_active], or NULL = every active
                               particle is a sink.  With flags, acc/pot are
                               written only for flagged particles (the others
                               are left untouched) and P2P is skipped for
                               leaves without a flagged particle; the flagged
                               results equal those without flags bit for bit.
                               Every active particle is still a source.  Read
                               by evaluations only.                          */
} fmm_request;

/* Build the trees and lists of n_req systems at once (sum of n_active <=
 * max_n).  Same rules and waiting behaviour as fmm_build. */
fmm_status fmm_build_batched(fmm_ctx *ctx, int n_req, const fmm_request *reqs, double eps,
                             double theta);

/* Evaluate the n_req systems of the last fmm_build_batched (same pos, active,
 * n_total, n_active in the same order, else FMM_ESTALE); masses and outputs
 * may differ from call to call, and a system with mass == NULL is skipped.
 * Asynchronous, like fmm_evaluate. */
fmm_status fmm_evaluate_batched(fmm_ctx *ctx, int n_req, const fmm_request *reqs, int p);

/* fmm_build_batched followed by fmm_evaluate_batched. */
fmm_status fmm_forces_batched(fmm_ctx *ctx, int n_req, const fmm_request *reqs, double eps,
                              double theta, int p);

/* Sizes of the current tree (all systems of a batch together): info[0]
 * n_active, [1] nodes, [2] unordered M2L
 * pairs, [3] unordered P2P leaf pairs (self pairs included), [4] depth,
 * [5] leaves, [6] ordered M2L entries, [7] ordered P2P entries, [8] ordered
 * particle-particle interactions evaluated by P2P. */
fmm_status fmm_tree_info(fmm_ctx *ctx, int64_t info[9]);

/* Builds of few active particles (all systems of a batch together) run as
 * two single-workgroup launches with one readback: enable = 1 (the default)
 * up to 1024 particles, beyond which the multi-workgroup path is faster;
 * enable = 2 up to 8192, the most those launches hold; enable = 0 never.
 * Trees, lists and results are the same either way (for comparison and
 * tests).  Other values: FMM_EINVAL. */
fmm_status fmm_set_small_path(fmm_ctx *ctx, int enable);

/* enable = 1: multi-workgroup builds queue the tree and the walk for the
 * deepest split level of the last four builds on this context, behind the
 * sort, and read the tree header once at the end (instead of after the
 * split-depth search, after the tree and after the walk); fmm_forces also
 * queues the evaluation before that read when the batch holds the same
 * systems as the last build within a quarter of its size.  A build whose
 * tree needs more levels, or whose workspace overflows, is redone the
 * classic way (and re-evaluated).  Trees, lists and forces are the same
 * either way.  enable = 0 (the default): the classic sequence.  Either call
 * forgets the recorded levels. */
fmm_status fmm_set_level_prediction(fmm_ctx *ctx, int enable);

/* Canonical host copy of the current tree, for comparison with other
 * implementations: nodes in pre-order (sorted by (begin, level)); perm[i] =
 * active slot of the i-th particle in Morton order; pairs as (a <= b) over
 * pre-order ids, sorted.  All outputs are HOST buffers sized from
 * fmm_tree_info; any pointer may be NULL.  Synchronises the stream.  Only for
 * a tree built from a single system (FMM_EINVAL otherwise). */
fmm_status fmm_export_tree(fmm_ctx *ctx, int64_t *perm, int32_t *level, uint64_t *prefix,
                           int64_t *begin, int64_t *end, int32_t *is_leaf, double *centre,
                           double *half, int64_t *m2l_pairs, int64_t *p2p_pairs, double *box);

/* Stream-ordered FP64 reductions over n particles (device SoA inputs, any may
 * be NULL): out[0..2] sum m a, out[3..5] sum m v, out[6..8] sum m x cross v,
 * out[9] kinetic energy, out[10] potential energy 0.5 sum m Phi,
 * out[11] sum m |a|.  out is a HOST array of 12 doubles; synchronises. */
fmm_status fmm_invariants(fmm_ctx *ctx, const double *pos, const double *vel, const double *mass,
                          const double *acc, const double *pot, int64_t n, double out[12]);

/* fmm_invariants for callers that cannot allocate device memory or wait for
 * the device: code under HIP graph capture, tight serving loops.  The same
 * twelve sums in the same order, bit for bit, but written to DEVICE memory
 * out[0..11] (caller-owned) on `stream` (a hipStream_t, NULL = the null
 * stream), without a context, an allocation, a copy or a synchronisation.
 * Inputs as for fmm_invariants (device SoA over n particles, any may be
 * NULL).  Its scratch is a library-owned device array of 512 x 12 doubles
 * (48 KiB on each device it runs on, kept until the process ends) whatever n
 * is, so no n is too large for it; every call on one device shares that
 * array, so calls that overlap on one device (different streams) race and
 * must be ordered by the caller.  FMM_EINVAL: out NULL or n < 0;
 * FMM_EDEVICE: the scratch could not be looked up or a launch failed. */
fmm_status fmm_invariants_noalloc(void *stream, const double *pos, const double *vel,
                                  const double *mass, const double *acc, const double *pot,
                                  int64_t n, double *out);

/* Per-phase timing with HIP events recorded on the context's stream between
 * launch groups (nothing else changes).  enable = 1 starts recording every
 * phase, enable = 2 only the M2L and P2P kernels (one event pair each per
 * evaluation, on the stream each runs on); both clear the totals; 0 stops. */
fmm_status fmm_profile_enable(fmm_ctx *ctx, int enable);

/* Totals since enabling: ms[k] milliseconds and calls[k] timed launch groups
 * of phase k: 0 root box + keys + radix sort, 1 tree split, 2 dual walk,
 * 3 P2M + M2M, 4 M2L, 5 P2P, 6 L2L + L2P (two groups per evaluation).
 * Waits for the recorded work. */
fmm_status fmm_profile_read(fmm_ctx *ctx, double ms[7], int64_t calls[7]);

/* ---------------------------------------------------------------------------
 * HHS integrator (Sec. 2.2, Algorithms 1-3)
 * ------------------------------------------------------------------------- */
typedef struct {
    double *pos;      /* device, 3 x n SoA, FP64 (updated in place)             */
    double *vel;      /* device, 3 x n SoA, FP64 (updated in place)             */
    const double *mass; /* device, n                                            */
    double *a_old;    /* device, n: |a| of the latest second kickS2F            */
    double *a_cur;    /* device, n: |a| of the latest second kickFS2S           */
    int32_t *rung;    /* device, n: timestep rung (0 = dt_top)                  */
    int64_t n;
    double t;         /* host-side time, advanced by hhs_step                    */
    double *a_tot;    /* device, n, or NULL: |a| due to all the mass, from the
                         full solve of hhs_init and then the second kickFS2S of
                         each top-level KDK (Eq. 9); needed when eta1 > 0      */
} hhs_state;

typedef struct {
    double eps, theta; /* as for fmm_build                                      */
    int p;             /* expansion order                                       */
    double eta;        /* timestep dt_i = sqrt(eta * eps / (|a_old| + |a_cur|))  */
    int max_levels;    /* rungs 0 .. max_levels-1 (>= 1)                         */
    int freeze_rungs;  /* nonzero: keep the rungs in state->rung                 */
    double eta1;       /* > 0: also dt_i <= sqrt(eta1 * eps / |a|_tot) (Eq. 9,
                          Sec. 3.4); 0: off                                     */
    const struct fmm_cosmo *cosmo; /* NULL, or the comoving form (Sec. 3.5):
                          state->t and dt_top are in ln a, velocities are
                          canonical momenta per unit mass, every kick and drift
                          is scaled by this table's factors (Eqs. 10-11) over
                          its own sub-interval instead of its length, and a
                          rung's step is compared in physical time, d(ln a)/H
                          at the start of the subsystem's step.  hhs_step and
                          hhs_step_batched only (trad_step and the server
                          reject it)                                           */
} hhs_params;

/* Full force solve on all n particles, then a_cur = |a|, a_old = 0 (and
 * a_tot = |a| when the state has that array). */
fmm_status hhs_init(fmm_ctx *ctx, hhs_state *st, const hhs_params *hp);

/* One top-level step of length dt_top (EVOLVE_HOLD at rung 0).  Rung of a
 * particle: the smallest r >= 0 with dt_top 2^-r <= dt_i (clamped to
 * max_levels-1), recomputed for a subsystem on entry when Algorithm 1 asks
 * for it.  At rung k the slow set is {rung <= k}, the fast set {rung > k}.
 * Each KDK (Algorithm 2) evaluates kickS2F (fast sinks, masses of the fast set
 * zeroed) and kickFS2S (slow sinks, all masses) on one tree built over the
 * joint set, each evaluation with the kicked set as its only sinks; a kick
 * with no sinks, or a kickS2F with an empty slow set, is skipped.  With
 * eta1 > 0 the rung must also give dt_top 2^-r <= sqrt(eta1 eps / |a|_tot):
 * the second kickFS2S of each top-level KDK is then evaluated at every
 * particle and refreshes a_tot (a top-level KDK with no slow particle skips
 * that kick and leaves a_tot as it was); FMM_EINVAL when eta1 > 0 and a_tot is
 * NULL, or eta1 < 0.  Kicks and drifts are FP64.  stats (host, may be NULL):
 * [0] force calls, [1] sum of active particles over the calls, [2] tree builds. */
fmm_status hhs_step(fmm_ctx *ctx, hhs_state *st, const hhs_params *hp, double dt_top,
                    int64_t stats[3]);

/* The paper's comparison integrator (Sec. 2.3): individual timesteps, each
 * force evaluation giving the active particles the acceleration due to all
 * the mass, with inactive particles where their last step left them (not
 * synchronised).  One top step of length dt_top on the state of hhs_step
 * (a_old is set to 0; a_cur holds |a| of each particle's latest evaluation):
 * an all-particle solve at the start gives a_cur and, unless freeze_rungs,
 * the rungs (the rule of hhs_step with |a| = a_cur); every particle takes the
 * opening half kick of its step dt_top 2^-rung; the top step is split into
 * 2^R ticks (R the deepest rung present); at the end of tick j the particles
 * with rung >= R - ctz(j+1) drift over their step, get the acceleration of a
 * solve over all particles at the stored positions, and take the closing half
 * kick and, before the last tick, the opening half kick of their next step (two
 * separate FP64 additions).  1 + 2^R force solves per call, each with a tree
 * over all particles and the particles of the tick as its only sinks.  stats (host, may be NULL): [0] solves, [1] sum over the solves
 * of the particles kicked with their result (n for the first), [2] tree
 * builds.  Synchronous: returns after the step has finished on the device.
 * FMM_EINVAL for bad parameters, a rung outside 0..max_levels-1 (frozen
 * rungs) or dt_top zero or not finite. */
fmm_status trad_step(fmm_ctx *ctx, hhs_state *st, const hhs_params *hp, double dt_top,
                     int64_t stats[3]);

/* Device scratch of one system's integration (rung split lists for every
 * rung, masked masses, accelerations): about hhs_run_bytes(n, max_levels)
 * bytes of device memory, owned by the run and freed by hhs_run_destroy
 * (which waits for the context's stream).  Serves systems of up to n
 * particles and max_levels rungs.  FMM_EINVAL for n < 1 or max_levels
 * outside 1..30, FMM_ENOMEM when the device is full (nothing kept). */
typedef struct hhs_run hhs_run;
int64_t hhs_run_bytes(int64_t n, int max_levels);
fmm_status hhs_run_create(fmm_ctx *ctx, int64_t n, int max_levels, hhs_run **out);
fmm_status hhs_run_destroy(hhs_run *run);

/* hhs_init for n_sys independent systems in one batched force solve; runs[i]
 * is the scratch of states[i] (distinct runs, distinct state arrays). */
fmm_status hhs_init_batched(fmm_ctx *ctx, int n_sys, hhs_run *const *runs,
                            hhs_state *const *states, const hhs_params *hp);

/* One top-level step of each of n_sys independent systems (dt_top[i] for
 * states[i], dt_top a HOST array), with the semantics of hhs_step.  The
 * systems advance together: whenever several wait on a KDK (Algorithm 2)
 * their trees are built in one fmm_build_batched and their kicks evaluated in
 * two fmm_evaluate_batched calls, so every system ends bit-identical to a
 * hhs_step of it alone.  The sum of the particles of systems that wait
 * together must fit max_n.  stats: [0] force evaluations summed over the
 * systems, [1] sum of active particles over them, [2] batched tree builds. */
fmm_status hhs_step_batched(fmm_ctx *ctx, int n_sys, hhs_run *const *runs,
                            hhs_state *const *states, const hhs_params *hp,
                            const double *dt_top, int64_t stats[3]);

/* ---------------------------------------------------------------------------
 * Request server: an ensemble of independent HHS simulations with continuous
 * batching (each request advances one system from t = 0 to t_end with the
 * integrator above).  Not thread safe: one host thread drives a server.
 * ------------------------------------------------------------------------- */
typedef struct fmm_server fmm_server;

typedef struct {
    int64_t arena_bytes; /* device memory for resident requests, allocated once */
    int max_slots;       /* at most this many requests resident at a time       */
    double dt_max;       /* cap on a request's top-level step                   */
} serve_params;

typedef struct {
    const double *pos;   /* HOST, 3 x n SoA initial positions                   */
    const double *vel;   /* HOST, 3 x n SoA initial velocities                  */
    const double *mass;  /* HOST, n                                             */
    int64_t n;           /* 1 .. max_n of the context                           */
    double t_end;        /* > 0                                                 */
    double *pos_out;     /* HOST, 3 x n: positions at t_end (written when done) */
    double *vel_out;     /* HOST, 3 x n: velocities at t_end                    */
} serve_request;

typedef struct {
    int64_t id, n;
    int64_t steps;           /* top-level steps taken                            */
    int64_t force_calls;     /* force evaluations of this request                */
    int64_t force_particles; /* sum of their active particles                    */
    double dt_top, t_end;
    double t_submit, t_admit, t_done; /* seconds on the server's clock           */
} serve_result;

/* Device bytes one resident request of n particles takes from the arena
 * (state arrays and integrator scratch); -1 for bad arguments. */
int64_t serve_footprint(int64_t n, int max_levels);

/* A server on ctx (whose stream and solver parameters it uses; max_n of the
 * context bounds a request's size and the particles solved in one batched
 * call) with one set of HHS parameters for all requests.  Allocates the arena
 * (FMM_ENOMEM if it does not fit). */
fmm_status serve_create(fmm_ctx *ctx, const hhs_params *hp, const serve_params *sp,
                        fmm_server **out);
fmm_status serve_destroy(fmm_server *srv);

/* Queue a request (arrival order is admission order).  The host arrays are
 * read when the request is admitted and the outputs written when it is done:
 * they must stay valid until serve_poll returns its result (or it is
 * cancelled).  FMM_ENOMEM if its footprint exceeds the whole arena.  *id is
 * the request's id. */
fmm_status serve_submit(fmm_server *srv, const serve_request *rq, int64_t *id);

/* One scheduling step: rounds of the batched HHS driver (Algorithms 1-3 of
 * Sec. 2.2) over the resident requests, for about 2 ms of host time or until
 * a request finishes or nothing is left to do.  Each round first admits
 * queued requests in order while a slot and arena space are free (uploading
 * them, with one batched initial force solve; a request's top-level step is
 * the largest sqrt(eta eps / |a_i|) at t = 0 rounded down to a power of two,
 * at most dt_max, and its last step is cut to end at t_end); then every
 * resident request advances until it needs the device, a request that ended
 * its top-level step begins the next one (or, at t_end, is retired: outputs
 * downloaded, arena space and slot freed), and either all pending split
 * counts are read back at once or all pending KDK halves are solved in shared
 * launches.  Requests at different points of their steps share launches;
 * none waits for another to end its step.  The last round's device work may
 * still run on the context's stream on return; a result handed out by
 * serve_poll is complete (its outputs written).  A result does not depend on
 * the other requests served with it.  Outputs (may be NULL): the resident and
 * queued counts after the step. */
fmm_status serve_step(fmm_server *srv, int *n_resident, int *n_queued);

/* Up to max_out finished requests, in completion order. */
fmm_status serve_poll(fmm_server *srv, serve_result *out, int max_out, int *n_out);

/* Drop a queued or resident request (no result); FMM_EINVAL if unknown. */
fmm_status serve_cancel(fmm_server *srv, int64_t id);

/* info[0] resident, [1] queued, [2] finished not yet polled, [3] arena bytes
 * in use, [4] arena bytes, [5] scheduling rounds run. */
fmm_status serve_info(const fmm_server *srv, int64_t info[6]);

#ifdef __cplusplus
}
#endif
#endif /* FMM355_H */

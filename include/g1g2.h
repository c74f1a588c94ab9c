/*
 * g1g2.h -- C ABI of the MI355X G1-G2 propagator.
 *
 * The library propagates the time-diagonal one-particle Green function
 * G1 = G^<(t) together with the correlated two-particle Green function
 * G2 = script-G(t) of the G1-G2 scheme (Joost, Schluenzen, Bonitz,
 * arXiv:2002.12717) within the Hartree-Fock generalized Kadanoff-Baym ansatz.
 *
 * Units and conventions (fixed by the paper, Sec. II):
 *   hbar = 1; fermions; G^< = i n with n the one-particle density matrix
 *   (eq:g-glsymm); the pair interaction w_ijkl multiplies
 *   1/2 c+_i c+_j c_l c_k in the Hamiltonian (eq:h).
 *
 * Memory layout of every array crossing this boundary: row-major, last index
 * fastest, complex numbers as interleaved (re, im) IEEE doubles (the layout of
 * C99 double complex and of torch.complex128).
 *   general basis (nb spin orbitals):  h0, G1: [nb][nb];  w, G2: [nb]^4
 *   Hubbard basis (nb sites):          h0, G1: [2][nb][nb] (spin up, spin down);
 *                                      G2 = G2^{up down up down}: [nb]^4
 *
 * Pointers are host memory unless G1G2_PTR_DEVICE is set in desc.flags (then
 * they are device pointers on the current HIP device, e.g. torch data_ptr()).
 * g1g2_rhs always takes device pointers.  Inputs are copied; the caller keeps
 * ownership of everything it passes.  The context owns all device memory it
 * allocates and frees it in g1g2_destroy.  All work is ordered on the stream
 * given to g1g2_init (NULL = the default stream); calls that return host data
 * (observables, get_state) synchronize that stream.
 *
 * Errors: every call returns a g1g2_status; nothing throws or aborts across
 * this boundary.  The text of the last error of a context is available from
 * g1g2_last_error.  A context is not thread-safe.
 */
#ifndef G1G2_H
#define G1G2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    G1G2_OK = 0,
    G1G2_EINVAL = -1,       /* bad argument, shape or flag                         */
    G1G2_ENOMEM = -2,       /* device allocation failed                            */
    G1G2_EDEVICE = -3,      /* HIP runtime error or no usable device               */
    G1G2_EUNSUPPORTED = -4, /* basis x selfenergy x precision not implemented      */
    G1G2_EDIVERGED = -5,    /* non-finite state or occupation outside [-0.5, 1.5]  */
    G1G2_ESTATE = -6        /* call not valid in the current state of the context  */
} g1g2_status;

/* Selfenergy closing the G2 equation:
 *   SOA: second Born, eq:result_eom_soa (source Psi^-).
 *   GW : eq:g2-eq-gw-pi (source Psi without exchange unless G1G2_GW_EXCHANGE).
 *   TPP: particle-particle T matrix, eq:g2-eq-tpp-lambda.
 *   TPH: particle-hole T matrix, eq:g2-eq-tph-lambda.
 *   DSL: dynamically screened ladder (Sec. VI): GW with exchange plus both
 *        T-matrix ladders, eq:g2-dsl-equation-pi-lambda.
 * Implemented: every selfenergy in both bases, single clusters and Hubbard
 * batches (Hubbard GW and DSL need ns <= 64 and at most 4 neighbours per
 * site).  Other combinations return G1G2_EUNSUPPORTED.  Hubbard GW and DSL
 * store three G2 channels, [3][ns]^4 in every G2 argument: up-down-up-down,
 * up-up-up-up, down-down-down-down (the spin of each slot attached to its
 * index, eq:g2-gw-hubbard1/2).  In the Hubbard basis DSL adds both ladders
 * to the up-down-up-down channel; they vanish on the equal-spin channels,
 * whose interaction pairs opposite spins, and the exchange form of the
 * source equals Psi there for the same reason.  The general-basis
 * GW, T-matrix and DSL closures cost one (nb^2 x nb^2 x nb^2) complex GEMM per
 * polarization or ladder and right-hand side.                                  */
typedef enum { G1G2_SOA = 0, G1G2_GW = 1, G1G2_TPP = 2, G1G2_TPH = 3, G1G2_DSL = 4 } g1g2_selfenergy;

/* GENERAL: arbitrary orthonormal basis with a four-index w (Sec. III.C).
 * HUBBARD: Fermi-Hubbard model with on-site U (Sec. III.D); h0 per spin may be
 *          any Hermitian matrix (hopping plus on-site potentials).
 * JELLIUM: uniform electron gas in plane waves (Sec. III.E); created with
 *          g1g2_jellium_init.                                                   */
typedef enum { G1G2_GENERAL = 0, G1G2_HUBBARD = 1, G1G2_JELLIUM = 2 } g1g2_basis;

/* FP64: every operation in binary64.
 * MIXED: general basis: the O(nb^5) and O(nb^6) tensor contractions run in
 *        binary32 on the matrix cores with binary64 accumulation across
 *        blocks.  Hubbard basis (no contractions): the G2 stage copies of the
 *        Runge-Kutta step (inputs of stages 2-4) are stored in binary32 and
 *        all arithmetic is binary64.  In both bases G1, the Runge-Kutta state
 *        and running sum, h^HF, the collision integral and all observables
 *        stay binary64, and g1g2_rhs evaluates in binary64.                    */
typedef enum { G1G2_FP64 = 0, G1G2_MIXED = 1 } g1g2_precision;

enum {
    G1G2_PTR_DEVICE = 1,    /* host-side pointer arguments are device pointers      */
    G1G2_GW_EXCHANGE = 2,   /* GW: use Psi^- instead of Psi (end of Sec. IV.B)      */
    /* Hubbard stage kernel (both set: EINVAL).  By default the slice kernel (a
     * work-group stages whole (i,j) slices of G2 in LDS) runs when the clusters
     * hold at least 2^20 G2 elements in all (counting GW's three channels),
     * else the row kernel (one wave per G2 row).  Both need ns <= 64 and at
     * most 4 neighbours per site, else the per-element kernel runs. */
    G1G2_HUB_ROW_KERNEL = 4,    /* Hubbard: row kernel whatever the size          */
    G1G2_HUB_SLICE_KERNEL = 8,  /* Hubbard: slice kernel whatever the size        */
    /* General-basis DSL: build the polarization and particle-hole
     * quasi-Hamiltonians (h^eps, h^ph) from w^- instead of w, i.e. with their
     * exchange terms.  eq:g2-dsl-equation builds them from w; Sec. VI equates
     * DSL with neglecting three-particle correlations, and against exact
     * diagonalization only the exchange form reaches that order (density
     * error O(w^4) instead of O(w^3)) in a general basis.  EUNSUPPORTED with
     * any other basis or selfenergy. */
    G1G2_DSL_EXCHANGE = 16,
    /* Jellium T matrices: the ladder transform with two rows per work-group
     * whatever nb (by default four, two only above 512 momenta, where four
     * would exceed 64 KB of LDS); the rows are independent, so the results are
     * the same.  For tests of the two-row form on grids the oracle can take. */
    G1G2_JEL_LAD_ROWS2 = 32
};

typedef struct {
    int32_t basis;          /* g1g2_basis                                          */
    int32_t selfenergy;     /* g1g2_selfenergy                                     */
    int32_t precision;      /* g1g2_precision                                      */
    int32_t flags;          /* bitwise OR of the flags above                        */
    int32_t nb;             /* general: spin orbitals; Hubbard: sites per spin      */
    double U;               /* Hubbard on-site interaction (ignored for general)   */
} g1g2_desc;

typedef struct {
    double t;               /* current time                                        */
    double N[2];            /* particle numbers Tr n (general: N[0], N[1] = 0)      */
    double E_kin;           /* Tr(h0 n), summed over spins                          */
    double E_mf;            /* Hartree-Fock interaction energy                      */
    double E_corr;          /* correlation energy -1/2 Re sum w_ijkl G2_klij        */
    double E_tot;           /* E_kin + E_mf + E_corr                                */
    double docc;            /* Hubbard: mean double occupation                      */
    double herm_resid;      /* max |G2_ijkl - conj(G2_klij)| / max |G2| (eq:Gsymm_b) */
    double exch_resid;      /* general: max |G2_ijkl - G2_jilk| / max |G2|
                               (eq:Gsymm_a); Hubbard: 0 (the exchange partner of
                               the stored up-down-up-down block is another block) */
    double imbalance;       /* Hubbard: (N_left - N_right) / N with left/right the
                               sites of negative/positive drive profile x_i
                               (g1g2_set_drive); 0 without a drive profile      */
    int32_t diverged;       /* 1 once the divergence guard has fired (for this
                               cluster, in g1g2_batch_observables)                 */
    int64_t step;           /* completed Runge-Kutta steps                          */
    int64_t diverged_step;  /* the first step at whose end the guard fired (the
                               count of completed steps then), -1 if it has not;
                               cleared by g1g2_set_state                          */
} g1g2_obs;

typedef struct g1g2_ctx g1g2_ctx;

/* Create a propagator.  h0 and G1_0 are required; w is required for the
 * general basis and ignored (may be NULL) for Hubbard; G2_0 = NULL means an
 * uncorrelated initial state (G2 = 0, eq:ini-g2 with n_ijkl factorized).
 * hip_stream is a hipStream_t owned by the caller (NULL = default stream).
 * Returns EINVAL for inconsistent shapes or a non-Hermitian h0, EUNSUPPORTED
 * for combinations that are not implemented (general nb > 64; Hubbard GW or
 * DSL with ns > 64 or more than 4 neighbours per site).                    */
g1g2_status g1g2_init(g1g2_ctx** out, const g1g2_desc* desc, const void* h0, const void* w,
                      const void* G1_0, const void* G2_0, void* hip_stream);

/* Jellium (uniform electron gas, Sec. III.E, Sec. IV.D) in a plane-wave basis
 * on a periodic momentum grid dims[3] = (Lx, Ly, Lz), momentum index
 * n = x + Lx (y + Ly z), components added modulo the grid (so momentum
 * conservation is exact in the finite basis); desc->nb = Lx Ly Lz <= 1024.
 * The pair interaction is eq:jellium-w-matrix in the convention of eq:h:
 * w = delta(k1 + k2 - k3 - k4) v[k1 - k3] between equal spins of each particle,
 * v[nb] a host array of reals with v[0] = 0 (the neutralizing background; the
 * Hartree term then vanishes), and eps[2][nb] (host, reals) the one-particle
 * energies per spin.  Layouts crossing this boundary:
 *   G1 = [2][nb] complex: the diagonal G^{<,s}_p (eq:jellium-g1);
 *   G2 = [3][nb][nb][nb] complex, blocks up-up, up-down, down-down, element
 *        [c][P][Pb][Q] = G2^{a b a b}_{(P-Q, a), (Pb+Q, b), (P, a), (Pb, b)}
 *        (eq:g2-def-jellium; down-up follows from eq:Gsymm_a).
 * G2_0 may be NULL (uncorrelated start).  Selfenergies SOA (eq:jellium-g2),
 * GW (eq:jellium-gwpi, Psi^- with G1G2_GW_EXCHANGE), TPP (eq:jellium-lambdapp)
 * and TPH (eq:jellium-lambdaph), the T matrices with Psi^- and the partner
 * conj(Lambda_{P-Q, Pb+Q, -Q}); they hold one more [3][nb]^3 buffer (the
 * ladder sums, 484 MB at 6x6x6).  FP64 or MIXED (binary32 G2 stage copies,
 * like the Hubbard basis).  Flags: G1G2_PTR_DEVICE, G1G2_GW_EXCHANGE,
 * G1G2_JEL_LAD_ROWS2.  EUNSUPPORTED for DSL; EINVAL for other flags, bad dims,
 * nb != Lx Ly Lz or v[0] != 0.  Every other call
 * works as for the other bases except set_h0, set_U, set_drive, set_switch, the
 * adjoint and the batch calls (EUNSUPPORTED or ESTATE).  Observables: N per
 * spin, E_kin = sum eps n, E_mf the Fock energy, E_corr.                    */
g1g2_status g1g2_jellium_init(g1g2_ctx** out, const g1g2_desc* desc, const int32_t* dims, const double* eps,
                              const double* v, const void* G1_0, const void* G2_0, void* hip_stream);

/* One evaluation of the right-hand side (dG1/dt, dG2/dt) of the closed system
 * eq:eom_gone-2 + eq:eom_gone-I + the G2 equation of the selfenergy, at time t
 * with the context's current h0, U and drive.  G1, G2 in, dG1, dG2 out: device
 * pointers in the layouts above.  Does not change the propagated state.     */
g1g2_status g1g2_rhs(g1g2_ctx* ctx, double t, const void* G1, const void* G2,
                     void* dG1, void* dG2);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): g1g2_rhs of
 * one Hubbard cluster that allocates nothing, copies nothing and does not
 * synchronize.  It reads G1, G2 and writes dG1, dG2 (device pointers, the
 * layouts above), ordered on the context's stream; the call returns before the
 * work completes.  The diagonal gathers of TPH, GW and DSL (2, 6 and 8 ns^3
 * complex elements) go to a static scratch array of 32 MiB per GPU (enough for
 * every closure up to ns = 64), held until the process ends and shared by every
 * call on that GPU: calls that overlap on one GPU race for it, so order them
 * (one stream, or events between streams).  The results equal g1g2_rhs.
 * EUNSUPPORTED for the general basis, ESTATE on a batch, EINVAL when the
 * gathers exceed the scratch (nothing is launched then).                     */
g1g2_status g1g2_rhs_noalloc(g1g2_ctx* ctx, double t, const void* G1, const void* G2,
                             void* dG1, void* dG2);

/* Advance the internal state by nsteps classical fourth-order Runge-Kutta
 * steps of size dt (h0(t) and U evaluated at the stage times).  The guard
 * checks G1 at the end of every step: a non-finite element or an occupation
 * outside [-0.5, 1.5] marks the cluster (the general basis is one cluster)
 * with the number of that step.  All nsteps steps still run; then the call
 * returns EDIVERGED, and g1g2_last_error names the first step and cluster
 * (g1g2_obs.diverged / diverged_step per cluster).  With a stream, whole
 * groups of 8 steps replay one captured HIP graph (captured at the first call
 * with 8 or more steps, again only when dt changes).                        */
g1g2_status g1g2_step_rk4(g1g2_ctx* ctx, double dt, int64_t nsteps);

/* Which kernels g1g2_step_rk4 uses for this context, as decided by the
 * library (sizes, selfenergy, flags, drive and switching ramp as they are
 * now): GENERAL (the general-basis matrix-core stages), HUB_PERSISTENT
 * (whole steps of one small Hubbard cluster in one work-group), HUB_SLICE,
 * HUB_ROW or HUB_ELEMENT (one launch per Runge-Kutta stage), JELLIUM.      */
enum {
    G1G2_PATH_GENERAL = 0,
    G1G2_PATH_HUB_PERSISTENT = 1,
    G1G2_PATH_HUB_SLICE = 2,
    G1G2_PATH_HUB_ROW = 3,
    G1G2_PATH_HUB_ELEMENT = 4,
    G1G2_PATH_JELLIUM = 5
};
g1g2_status g1g2_step_path(const g1g2_ctx* ctx, int32_t* path);

/* Capture now the HIP graph of 8 steps of size dt that g1g2_step_rk4
 * replays, so that no later call pays for the capture (before a timed or
 * latency-bound loop).  Returns OK and does nothing when steps are not
 * replayed from graphs: no stream given, a drive or switching ramp set, or
 * the persistent small-cluster kernel takes the steps.  EINVAL for dt <= 0. */
g1g2_status g1g2_prepare_graph(g1g2_ctx* ctx, double dt);

/* Observables of the current state; synchronizes the stream. */
g1g2_status g1g2_observables(g1g2_ctx* ctx, g1g2_obs* out);

/* Hubbard only: site-resolved densities n^up_ii, n^dn_ii and double
 * occupations n^up_ii n^dn_ii - Re G2_iiii (host arrays of nb doubles).   */
g1g2_status g1g2_site_observables(g1g2_ctx* ctx, double* n_up, double* n_dn, double* docc);

/* Copy the current state out / in (layouts above; G2 may be NULL on get). */
g1g2_status g1g2_get_state(g1g2_ctx* ctx, void* G1, void* G2, double* t);
g1g2_status g1g2_set_state(g1g2_ctx* ctx, const void* G1, const void* G2, double t);

/* Replace the one-particle Hamiltonian (same layout and sparsity rules as in
 * g1g2_init); used for excitations between calls of g1g2_step_rk4.         */
g1g2_status g1g2_set_h0(g1g2_ctx* ctx, const void* h0);

/* Hubbard: change the on-site interaction U. */
g1g2_status g1g2_set_U(g1g2_ctx* ctx, double U);

/* Hubbard: time-dependent on-site drive added to h0 for both spins,
 *   v_i(t) = sum_{m<M} c_m exp(-(t - t_center_m)^2 / (2 tau^2)) x_i.
 * Host arrays x[nb], c[M], t_center[M]; M = 0 removes the drive.            */
g1g2_status g1g2_set_drive(g1g2_ctx* ctx, const double* x, int32_t M, const double* c,
                           const double* t_center, double tau);

/* Adiabatic switching of the interaction (both bases, single clusters and
 * Hubbard batches): the preparation of a correlated initial state by turning
 * the interaction on slowly from an uncorrelated start (Sec. III.F and the
 * outlook of Sec. VIII).  The interaction becomes U(t) = U phi(t) (every
 * cluster) or w(t) = w phi(t) (general basis) with
 *   phi = 0 for t <= t_on, sin^2(pi x / 2) with x = (t - t_on) / tau during
 *   the ramp, and 1 for t >= t_on + tau,
 * evaluated at every Runge-Kutta stage time; the observables use U(t) at the
 * state's time.  tau = 0 switches it off (U constant).  Steps are not
 * graph-captured while a ramp is set, and the adjoint refuses it (its
 * gradient assumes a constant U).  EINVAL for tau < 0 or non-finite values. */
g1g2_status g1g2_set_switch(g1g2_ctx* ctx, double t_on, double tau);

/* Ragged batch of independent Hubbard clusters (configurations of uneven
 * size and U) propagated together: every Runge-Kutta stage of the whole batch
 * is one kernel launch over a flat work list, and g1g2_step_rk4 replays
 * captured HIP graphs of whole steps when a stream is given.  desc supplies
 * basis (HUBBARD), selfenergy (any) and precision (FP64 or MIXED); per cluster
 * c: ns[c] sites, on-site U[c], h0[c] and G1_0[c] as host arrays
 * [2][ns][ns]; G2(0) = 0.  chunk[c] sets the G2 elements handled by one
 * work-group of cluster c (NULL or 0: default), e.g. from an autotuning
 * table: chunk > 0 is, for the slice kernel, the most G2 elements one work
 * item stages (whole (i,j) slices, at least one, at most 4096 elements), and,
 * for the row kernel, the granularity of its work (one wave per G2 row
 * A[i][j][k][:], rounded to whole wave units of rows); chunk < 0 selects the
 * per-element kernel with |chunk| elements per work-group (any negative entry
 * selects the per-element kernel for the whole batch).
 * g1g2_step_rk4, g1g2_profile and g1g2_destroy act on the whole batch; the
 * single-cluster calls (rhs, get/set_state, set_h0/U/drive) return ESTATE. */
g1g2_status g1g2_batch_init(g1g2_ctx** out, const g1g2_desc* desc, int32_t n, const int32_t* ns,
                            const double* U, const void* const* h0, const void* const* G1_0,
                            const int32_t* chunk, void* hip_stream);
/* Observables of every cluster: out[n] (herm_resid is not computed). */
g1g2_status g1g2_batch_observables(g1g2_ctx* ctx, g1g2_obs* out);
/* State of one cluster into host arrays G1 [2][ns][ns] and (if not NULL) G2
 * [nchan][ns]^4 (three channels for GW and DSL, one otherwise). */
g1g2_status g1g2_batch_get_state(g1g2_ctx* ctx, int32_t cluster, void* G1, void* G2);

/* Discrete adjoint of the Runge-Kutta propagation (single-cluster Hubbard,
 * SOA, with or without drive; binary64, or MIXED: the forward pass and its
 * recomputed segments keep the G2 stage copies in binary32 like the mixed
 * stages of g1g2_step_rk4, and the reverse sweep reads them as such, with
 * every cotangent and sum in binary64).  g1g2_forward_checkpointed advances the state
 * by nsteps steps of size dt exactly like g1g2_step_rk4 and keeps a device
 * copy of the state every `interval` steps (interval <= 0:
 * ceil(sqrt(nsteps / 4))); g1g2_adjoint recomputes one segment at a time and
 * keeps its states and Runge-Kutta stage states, so device memory grows by
 * about (nsteps/interval + 4 interval + 8) states (a state of ns = 64 is
 * 268 MB: 4000 steps hold about 70 GB).
 * g1g2_adjoint then returns the loss
 *   L = sum_i a[i] d_i(T) + sum_i b[i] (n^up_ii(T) + n^dn_ii(T)),
 *   n_ii = Im G^<_ii,  d_i = n^up_ii n^dn_ii - Re G2_iiii,
 * and its exact derivatives with respect to the drive coefficients c_m
 * (grad_c[M], M as given to g1g2_set_drive; may be NULL) and U (grad_U),
 * by the reverse sweep of the discrete RK4 map with each checkpoint segment
 * recomputed once.  a, b: host arrays of nb doubles.  The final state is left
 * in place.  ESTATE without a preceding forward_checkpointed;
 * EUNSUPPORTED for other bases, selfenergies or batches, and with a
 * switching ramp set.                                                       */
g1g2_status g1g2_forward_checkpointed(g1g2_ctx* ctx, double dt, int64_t nsteps, int32_t interval);
g1g2_status g1g2_adjoint(g1g2_ctx* ctx, const double* a, const double* b, double* grad_c,
                         double* grad_U, double* loss);

/* Profiling aid.  Runs nsteps Runge-Kutta steps of size dt exactly like
 * g1g2_step_rk4 (advancing the state), or, for nsteps = 0, one right-hand-side
 * evaluation of the current state, with a HIP event recorded on the context's
 * stream after every kernel launch.  For each distinct kernel k (at most
 * max_kernels, the number in *count) it returns the summed time between the
 * event before and after its launches, ms_total[k], and the number of
 * launches, launches[k]; g1g2_profile_name(ctx, k) names the kernel.
 * Synchronizes the stream.                                                  */
g1g2_status g1g2_profile(g1g2_ctx* ctx, double dt, int64_t nsteps, int32_t max_kernels,
                         double* ms_total, int32_t* launches, int32_t* count);
const char* g1g2_profile_name(const g1g2_ctx* ctx, int32_t k);
/* The same per-kernel timing for one reverse sweep of g1g2_adjoint with the
 * loss weights a, b (after g1g2_forward_checkpointed; the gradients are not
 * returned, the final state is left in place).  Errors as g1g2_adjoint.     */
g1g2_status g1g2_profile_adjoint(g1g2_ctx* ctx, const double* a, const double* b, int32_t max_kernels,
                                 double* ms_total, int32_t* launches, int32_t* count);

void g1g2_destroy(g1g2_ctx* ctx);
const char* g1g2_strerror(g1g2_status status);
const char* g1g2_last_error(const g1g2_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* G1G2_H */

/*
 * lbm.h - C ABI of the MI355X lattice-Boltzmann step of the grand-potential
 * phase-field model of a two-phase ternary fluid (Verdier, Cartalade & Plapp,
 * arXiv 2409.03401).
 *
 * One simulation domain on one GPU.  Every device buffer is owned by the
 * caller; the library never allocates device memory.  All calls are
 * asynchronous on the HIP stream passed as `stream` (a hipStream_t; NULL is the
 * default stream) unless stated otherwise.  Errors: a call returns LBM_OK (0)
 * or a negative LBM_E* code and leaves a message for lbm_last_error() (per
 * host thread).  No C++ exception crosses this interface.
 *
 * Grids are indexed node = (z * ny + y) * nx + x, x fastest.  In 2D nz = 1.
 * Same inputs give bitwise-identical outputs (no floating-point atomics).
 */
#ifndef LBM_GP_TERNARY_H
#define LBM_GP_TERNARY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------------- */
#define LBM_OK 0
#define LBM_EINVAL (-1)       /* bad argument or inconsistent configuration        */
#define LBM_ESIZE (-2)        /* a caller buffer is smaller than required          */
#define LBM_EUNSTABLE (-3)    /* a BGK rate lies outside (0, 2) (tau <= 0)         */
#define LBM_EUNSUPPORTED (-4) /* lattice / precision / boundary combination        */
#define LBM_EHIP (-5)         /* a HIP runtime call failed                         */

/* ---- configuration values --------------------------------------------------- */
#define LBM_NONE 0            /* no flow: u = 0, no f populations                  */
#define LBM_D2Q9 9            /* fluid lattices, Tables tab:D2Q9 / tab:D3Q19; also */
#define LBM_D3Q19 19          /* the paper's scalar lattices                       */
#define LBM_D2Q5 5            /* reduced scalar lattices for phi, c^A, c^B         */
#define LBM_D3Q7 7

/* collision operators (Section 3).  LBM_BGK is the paper's single-rate collision.
 * LBM_TRT, the two-relaxation-time alternative Section 3 names, relaxes the part
 * of X_k - X_k^eq that is symmetric over (k, opp(k)) at w+ and the antisymmetric
 * part at w- (the equilibria keep their -F_k/2, -G_k/2 shifts and the sources are
 * added as in BGK).  The transport coefficient sets one rate as in BGK: the
 * viscosity sets w+ of f, the mobilities set w- of g, h^A, h^B; the other follows
 * from the magic parameter Lambda = (1/w+ - 1/2)(1/w- - 1/2) (trt_magic; 3/16
 * puts half-way bounce-back walls exactly at the half link).  Any storage
 * precision, no adjoint. */
#define LBM_BGK 0
#define LBM_TRT 1
/* LBM_MRT, the multiple-relaxation-time alternative Section 3 names: X - X^eq is
 * taken to a moment basis orthogonal in sum_k w_k a_k b_k (Gram-Schmidt over the
 * polynomials 1, c, |c|^2, the traceless second order, then third and fourth
 * order), each moment relaxed at its own rate, and taken back; sources as in BGK.
 * f: the traceless second order at the viscous rate, the trace (bulk), third and
 * fourth orders at mrt_rates[0][0..2], orders 0 and 1 conserved.  g, h^A, h^B: the
 * first order (diffusive flux) at the mobility rate, orders 0 and 2 at
 * mrt_rates[1][0], third and fourth at mrt_rates[1][1..2].  Rates in (0, 2);
 * any storage precision, Boussinesq, no adjoint. */
#define LBM_MRT 2

/* general_kappa = 1 (any storage precision, BGK, Boussinesq, no adjoint): the
 * quadratic free energies of Eq. Taylor with full curvature matrices K_pi, given
 * as kappa_pi = K (K_pi)^-1 (symmetric positive definite; the identity is the
 * paper's model).  The grand potentials become -1/2 mu.kappa_pi mu - mu.c_pi^eq,
 * so the closure is c = c^eq(phi) + kappa(phi) mu with kappa(phi) = kappa_0 +
 * p(phi) (kappa_1 - kappa_0), solved for mu per node (2 x 2), Delta omega gains
 * -1/2 mu.(kappa_0 - kappa_1) mu, and the free-energy diagnostic uses
 * 1/2 mu.kappa(phi) mu.  lbm_init takes mu_0 and derives c from this closure. */

/* variable_density = 1 (needs a fluid lattice; any storage precision, no adjoint):
 * the high-density-ratio form Section 3 names after Eq. Velocity.  rho(phi) =
 * rho0 + drho phi enters the inertia; f holds dimensionless populations with
 * zeroth moment p* = p_h / (rho c_s^2) and equilibrium w_k [p* + c_k.u / c_s^2 +
 * (c_k.u)^2 / (2 c_s^4) - u.u / (2 c_s^2)] - F_k / 2, F_k the forcing population
 * divided by rho c_s^2; the pressure force -p* c_s^2 grad rho and the viscous
 * force -(nu w+ / c_s^2) Pi . grad rho (Pi the second moment of f - f^eq at the
 * predictor velocity sum_k f_k c_k + (F_s + F_b + F_p) / (2 rho)) join the total
 * force.  Buoyancy stays (phi - phi_ref) drho g.  lbm_moments reports p_h. */

/* ncomp = 3 (D2Q5 / D3Q7 scalar lattices, BGK, Boussinesq, any storage precision,
 * no adjoint): the N-component extension the conclusion names, with one more
 * independent composition C (four components) and the same quadratic free energies
 * (Eq. Taylor, unit curvatures).  C has its own h^C populations and mobility M_C;
 * the closure of Eq. PotChem holds for each composition, and Delta omega =
 * -sum_alpha mu^alpha (c_0 - c_1)^alpha runs over A, B, C.  Initialise with
 * lbm_init_multi; populations are ordered f, g, hA, hB, hC. */

#define LBM_PERIODIC 0
#define LBM_WALLS 1           /* half-way bounce-back walls at both ends of an axis */

#define LBM_FP64 0            /* FP64 storage and arithmetic                        */
#define LBM_FP32 1            /* FP32 storage and arithmetic                        */
#define LBM_FP32_FP16STORE 2  /* FP32 arithmetic, moving populations stored in FP16 */
#define LBM_FP32_BF16STORE 3  /* FP32 arithmetic, moving populations stored in BF16 */

#define LBM_OUT_F64 0
#define LBM_OUT_F32 1

/* moment masks for lbm_moments; out[i] belongs to the i-th bit */
#define LBM_M_PHI (1u << 0)   /* phase field, Eq. Moment0_Phi                       */
#define LBM_M_CA (1u << 1)    /* compositions, Eq. Moment0_c_alpha                  */
#define LBM_M_CB (1u << 2)
#define LBM_M_MUA (1u << 3)   /* diffusion potentials, Eq. PotChem                  */
#define LBM_M_MUB (1u << 4)
#define LBM_M_P (1u << 5)     /* hydrodynamic pressure, Eq. HydroPressure           */
#define LBM_M_UX (1u << 6)    /* velocity, Eq. Velocity                             */
#define LBM_M_UY (1u << 7)
#define LBM_M_UZ (1u << 8)
#define LBM_M_CC (1u << 9)    /* c^C and mu^C of a third composition (ncomp = 3)    */
#define LBM_M_MUC (1u << 10)
#define LBM_NMOM 11

/* diagnostics written by lbm_diagnostics, in this order */
#define LBM_D_SUM_CA 0        /* sum_x c^A                                          */
#define LBM_D_SUM_CB 1        /* sum_x c^B                                          */
#define LBM_D_SUM_PHI 2       /* sum_x phi                                          */
#define LBM_D_KINETIC 3       /* sum_x rho |u|^2 / 2 (rho0, or rho(phi) if variable) */
#define LBM_D_MAX_U 4         /* max_x |u|                                          */
#define LBM_D_INTERFACE 5     /* sum_x (4/W) phi (1 - phi), integrand of Eq. Rmoy_2D */
#define LBM_D_FREE_ENERGY 6   /* sum_x [W^2/2 |grad phi|^2 + omega_dw + lambda/2 |mu|^2] */
#define LBM_D_NAN_COUNT 7     /* nodes whose phi or a composition is not finite     */
/* Section 4.2.2, geometry measurements.  LBM_D_DROPLETS is the Euler
 * characteristic of the union of the closed unit cells of the nodes with
 * phi >= 1/2 (vertices - edges + faces - cubes; periodic axes close on a torus,
 * cells end at walls), which is the droplet count N for separated simply
 * connected droplets.  The count runs over the axes of the run: 2D runs and 3D
 * runs with nz = 1 give a planar complex.  LBM_D_MEAN_RADIUS is <R> from the
 * interface integral I = LBM_D_INTERFACE: I / (2 pi N) in 2D (Eq. Rmoy_2D),
 * sqrt(I / (4 pi N)) in 3D (spheres), 0 when N <= 0. */
#define LBM_D_DROPLETS 8
#define LBM_D_MEAN_RADIUS 9
#define LBM_D_SUM_CC 10       /* sum_x c^C (ncomp = 3; 0 otherwise)                 */
#define LBM_NDIAG 11

/*
 * Physical parameters in lattice units (dx = dt = 1).  Section 2 of the paper
 * for the model, Section 3 for the lattices; [2] arrays are (phase 0, phase 1),
 * c_eq[phase][component].
 */
typedef struct lbm_config {
    int32_t dim;               /* 2 or 3, or 0 to take it from the scalar lattice   */
    int32_t nx, ny, nz;        /* nz = 1 for 2D                                     */
    int32_t fluid;             /* LBM_NONE, LBM_D2Q9 (2D) or LBM_D3Q19 (3D)         */
    int32_t scalar;            /* LBM_D2Q5 / LBM_D2Q9 (2D), LBM_D3Q7 / LBM_D3Q19 (3D) */
    int32_t bc[3];             /* per axis x, y, z: LBM_PERIODIC or LBM_WALLS       */
    int32_t precision;         /* LBM_FP64 ... LBM_FP32_BF16STORE                   */
    int32_t gravity_mean_subtract; /* 1: buoyancy uses phi - <phi> of the previous
                                      step (for fully periodic boxes); 0: phi       */
    double W;                  /* interface width                                   */
    double lambda;             /* coupling constant K/H                             */
    double M_phi;              /* scaled phase-field mobility W^2 / tau_phi         */
    double M_A[2], M_B[2];     /* scaled species mobilities per phase               */
    double c_eq[2][2];         /* equilibrium compositions [phase][A|B]             */
    double rho0;               /* reference density                                 */
    double drho;               /* density difference (phase 1 denser)               */
    double g[3];               /* gravity                                           */
    double sigma;              /* surface tension                                   */
    double nu[2];              /* kinematic viscosity per phase                     */
    double store_ref[4];       /* 16-bit storage: reference per field f, g, hA, hB:
                                  moving population k is stored as the deviation
                                  x - w_k store_ref[F], rounded to nearest even;
                                  hA, hB must be 0 (w_k mu is near zero), and so
                                  must f with BF16 storage                          */
    int32_t store_shift[4];    /* FP16 storage: the deviation is scaled by
                                  2^store_shift[F] before rounding (FP16's range);
                                  BF16 (FP32's exponent range) ignores it           */
    int32_t collision;         /* LBM_BGK (the paper's, 0) or LBM_TRT               */
    int32_t variable_density;  /* 0: Boussinesq (the paper's); 1: rho(phi) model    */
    double trt_magic[2];       /* LBM_TRT: Lambda of f and of g, h^A, h^B (> 0)     */
    int32_t general_kappa;     /* 0: the paper's K_pi = K identity; 1: kappa below  */
    int32_t ncomp;             /* independent compositions: 0 or 2 (A, B: the
                                  paper's ternary fluid) or 3 (A, B, C)             */
    double kappa[2][3];        /* per phase (k_AA, k_AB, k_BB) = K (K_pi)^-1        */
    double mrt_rates[2][3];    /* LBM_MRT: f (bulk, 3rd, 4th), scalars (2nd, 3rd, 4th) */
    double c_eq_C[2];          /* ncomp = 3: equilibrium c^C per phase              */
    double M_C[2];             /* ncomp = 3: scaled mobility of C per phase         */
    int32_t store_shift_C;     /* ncomp = 3, FP16 storage: shift of h^C (reference 0) */
    int32_t reserved;          /* 0                                                 */
} lbm_config;

typedef struct lbm_handle lbm_handle;

/* Size of the state buffer lbm_init needs (two population copies, a small
 * reduction area and a one-byte-per-node mask of the diagnostics), and of one
 * checkpoint written by lbm_save.
 * Two copies, not an in-place (AA-pattern) layout: a step reads one copy and
 * writes the other, because each work-group recomputes phi on a one-node ring
 * from populations its neighbours are updating in the same launch; in place,
 * those reads would race with the neighbours' writes unless phi took a pass of
 * its own.  The cost is memory: twice the stored population bytes per node
 * (2 x 88 B with D3Q19 + 3 x D3Q7 and 16-bit storage, 23.8 GB for 512^3).
 * Tuning only: the environment variables LBM_TILE ("64x4" or "32x8" in 3D; "64x1",
 * "128x1" or "256x1" in 2D) and LBM_ZC (planes per work-group) override the launch
 * geometry the library chooses.  They are read whenever a configuration is checked,
 * so lbm_state_bytes and lbm_init must see the same values. */
int lbm_state_bytes(const lbm_config* cfg, size_t* bytes);
int lbm_checkpoint_bytes(const lbm_config* cfg, size_t* bytes);

/*
 * Initialise the populations at rest (Section 4.2.1): from the FP64 device
 * fields phi0, muA0, muB0 ([node]), compositions follow Eq. species_closure,
 * u = 0, p_h = 0, and every population is set to its equilibrium (Eqs. Feq,
 * Geq, Heq) including the -F_k/2 and -G_k/2 shifts.  `state` is a device
 * buffer of at least lbm_state_bytes; it must stay allocated until
 * lbm_destroy.  On success *out receives a host handle (owns no device memory).
 */
int lbm_init(const lbm_config* cfg, void* state, size_t state_bytes,
             const double* phi0, const double* muA0, const double* muB0,
             void* stream, lbm_handle** out);

/* As lbm_init, but with the compositions given instead of derived from the
 * closure: the device fields cA0, cB0 ([node], FP64) set the zeroth moments of
 * h^A, h^B while muA0, muB0 enter the equilibria and the source S.  This is the
 * initial condition of Section 4.2.1 (Eq. Compos_Init: c stepped at phi = 1/2,
 * mu = 0 everywhere), which is not in equilibrium with the closure.  NULL cA0 or
 * cB0: LBM_EINVAL. */
int lbm_init_composition(const lbm_config* cfg, void* state, size_t state_bytes,
                         const double* phi0, const double* cA0, const double* cB0,
                         const double* muA0, const double* muB0, void* stream, lbm_handle** out);

/* Initialisation for any number of compositions (ncomp of the configuration, 2 or
 * 3): as lbm_init with mu0[a] the FP64 device potential of composition a (A, B, C),
 * or, when c0 is not NULL, as lbm_init_composition with c0[a] its composition.  mu0
 * (and c0 when given) are host arrays of ncomp device pointers.  lbm_init and
 * lbm_init_composition return LBM_EINVAL for ncomp = 3. */
int lbm_init_multi(const lbm_config* cfg, void* state, size_t state_bytes, const double* phi0,
                   const double* const* mu0, const double* const* c0, void* stream, lbm_handle** out);

/* Advance nsteps >= 0 time steps (Section 3: moments, forces, BGK collision of
 * f, g, h^A, h^B, streaming with periodic or bounce-back boundaries). */
int lbm_step(lbm_handle* h, int64_t nsteps, void* stream);

/* Write the macroscopic fields of the current state into out[i] for each bit
 * i set in mask (device arrays of nx*ny*nz elements, LBM_OUT_F64 or
 * LBM_OUT_F32).  Entries of out for unset bits are ignored.  In 2D, uz is 0.
 * LBM_M_CC and LBM_M_MUC need ncomp = 3 (LBM_EINVAL otherwise). */
int lbm_moments(lbm_handle* h, uint32_t mask, void* const* out, int32_t out_dtype,
                void* stream);

/* FP64 reductions of the current state into host_out[LBM_NDIAG].  Synchronises
 * `stream`. */
int lbm_diagnostics(lbm_handle* h, double* host_out, void* stream);

/* Time series of the diagnostics (droplet count, mean radius and max |u| curves
 * of Sections 4.2.2-4.2.4): records lbm_diagnostics of the current state, then
 * advances `every` steps and records again, nsteps / every times.  host_out
 * receives (nsteps / every + 1) rows of LBM_NDIAG doubles.  nsteps >= 0 must be a
 * multiple of every >= 1 (LBM_EINVAL otherwise, nothing done).  Synchronises
 * `stream` at every record. */
int lbm_run_series(lbm_handle* h, int64_t nsteps, int64_t every, double* host_out, void* stream);

/* Current populations decoded to FP64, canonical order: f_0..f_{Qf-1},
 * g_0..g_{Qs-1}, hA_0.., hB_0.. (, hC_0..) (paper's direction order), each [node].
 * dst holds (Qf + (1 + ncomp) Qs) * nodes doubles.  set_populations encodes such an
 * array into the current state (rounding to the storage type). */
int lbm_get_populations(lbm_handle* h, double* dst, void* stream);
int lbm_set_populations(lbm_handle* h, const double* src, void* stream);

/* Checkpoint / resume: byte copy of the current population copy plus the
 * buffered <phi> of the gravity reference (the remaining bytes of the last 256
 * are zero, as is the padding after each slot, so equal states give equal
 * checkpoints byte for byte).  restore(save(s)) continues bitwise identically. */
int lbm_save(lbm_handle* h, void* dst, void* stream);
int lbm_restore(lbm_handle* h, const void* src, void* stream);

/* Restore a checkpoint (lbm_save layout, lbm_checkpoint_bytes) as the current state:
 * a device-to-device copy of the populations and the buffered <phi>, the same as
 * lbm_restore.  Used by a checkpointed adjoint to return to a stored state. */
int lbm_set_state(lbm_handle* h, const void* src, void* stream);

/* One step from the checkpoint `src` into the checkpoint `dst` (both laid out
 * as lbm_save writes them; lbm_checkpoint_bytes each), without touching the
 * handle's own copies.  It writes the populations and the buffered <phi> of
 * `dst`; the padding bytes of `dst` keep what they held (zero for a buffer that
 * lbm_save wrote).  When phi_src is not NULL it receives phi of `src`
 * (Eq. Moment0_Phi, [node], FP64 for LBM_FP64 storage, FP32 otherwise), the
 * field the step's stencil used.  Used to recompute states for the adjoint. */
int lbm_step_external(lbm_handle* h, const void* src, void* dst, void* phi_src, void* stream);

/* phi of the checkpoint `state` into `phi` ([node], same type as above). */
int lbm_phase_field(lbm_handle* h, const void* state, void* phi, void* stream);

/*
 * Discrete adjoint (reverse mode) of the step, for a loss L of the final phase
 * field.  The adjoint of a state is dL/dX_k(x) for its arriving populations
 * (Section 3); it lives in the caller's device workspace (`work`, `adj_inout`,
 * `adj_state0`: one buffer of lbm_adjoint_bytes holding two FP32 copies of the
 * adjoint populations, scratch rows, phi of a state and FP64 parameter partials).
 * The handle records which adjoint copy is current, so a workspace is used with the
 * handle that seeded it.  Supported for LBM_FP32 and LBM_FP64 storage with the
 * paper's BGK Boussinesq model (either scalar lattice), without
 * gravity_mean_subtract; other
 * configurations (TRT, MRT, variable density, general curvatures) return
 * LBM_EUNSUPPORTED.
 * Calls that share one workspace must not overlap.
 *
 *   lbm_adjoint_seed  : start from dL/dphi_T (FP64 device [node]) at the final
 *                       state `state` (a checkpoint, lbm_save layout), through
 *                       phi of Eq. Moment0_Phi with its predictor.  Clears the
 *                       parameter partials.
 *   lbm_adjoint_step  : adjoint of the step n -> n + 1 (Section 3 in reverse):
 *                       state_n is the checkpoint of state n (before the step,
 *                       lbm_save layout); the adjoint of state n + 1 held in the
 *                       workspace adj_inout becomes that of state n; the parameter
 *                       gradient collected so far (this step, and a seed before it)
 *                       is added to grad_params[6] (FP64 device, the order of
 *                       lbm_adjoint_theta).  phi of state n is computed into the
 *                       workspace first.
 *   lbm_adjoint_step_phi : the same step with phi of state n given (from
 *                       lbm_step_external or lbm_phase_field, so a recompute pass
 *                       need not form it twice); its parameter gradient stays in the
 *                       workspace for lbm_adjoint_theta.
 *   lbm_init_adjoint  : adjoint of lbm_init with mu_0 held fixed (Eqs. Geq, Heq,
 *                       species_closure, with the -S_0/2 and -F_0/2 shifts): from the
 *                       adjoint of state 0 in adj_state0 writes dL/dphi_0 (FP64
 *                       device [node]) and adds the remaining parameter gradient to
 *                       grad_params[6].  Uses the phi0, muA0, muB0 fields given to
 *                       lbm_init, which must still hold them; a handle made by
 *                       lbm_init_composition returns LBM_EUNSUPPORTED.
 *   lbm_adjoint_init  : adjoint of lbm_init with mu_0 held fixed: writes dL/dphi_0
 *                       (FP64 device [node]); phi0, muA0, muB0 as given to lbm_init.
 *   lbm_adjoint_theta : writes grad_theta[6] (FP64 device) = dL/d(M_phi, M^A_0,
 *                       M^A_1, M^B_0, M^B_1, W) accumulated in the workspace since
 *                       the last seed, set, lbm_adjoint_step or lbm_init_adjoint
 *                       (Eqs. SourceTerm_Phi, LBE_Phi, LBE_c_alpha,
 *                       SurfaceTension_Force and the mobility interpolation).
 *   lbm_adjoint_get / lbm_adjoint_set : the current adjoint as FP64 [slot][node]
 *                       in the canonical slot order of lbm_get_populations; set
 *                       also clears the parameter partials.
 */
int lbm_adjoint_bytes(const lbm_config* cfg, size_t* bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): lbm_adjoint_step without the
 * workspace's scratch part.  adj_state holds only the adjoint state: two FP32 copies
 * of Q_tot = Q_f + 3 Q_s adjoint slots followed by three FP32 rows of c_F, each slot
 * and row round_up(4 nodes, 256) bytes (the leading part of an lbm_adjoint_bytes
 * workspace, so one seeded by lbm_adjoint_seed or lbm_adjoint_set may be passed).
 * The per-step scratch (about 36 bytes per node) is a 32 MiB device array inside the
 * library, one per GPU, held until the process ends; larger grids return LBM_ESIZE.
 * The call allocates nothing.  The gradient of this step alone is added to
 * grad_params[6].  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (other streams, other threads) race. */
int lbm_adjoint_step_noalloc(lbm_handle* h, const void* state_n, void* adj_state, double* grad_params,
                             void* stream);
int lbm_adjoint_seed(lbm_handle* h, const void* state, const double* dL_dphi, void* work, void* stream);
int lbm_adjoint_step(lbm_handle* h, const void* state_n, void* adj_inout, double* grad_params, void* stream);
int lbm_adjoint_step_phi(lbm_handle* h, const void* state, const void* phi, void* work, void* stream);
int lbm_init_adjoint(lbm_handle* h, const void* adj_state0, double* grad_phi0, double* grad_params, void* stream);
int lbm_adjoint_init(lbm_handle* h, const double* phi0, const double* muA0, const double* muB0, void* work,
                     double* grad_phi0, void* stream);
int lbm_adjoint_theta(lbm_handle* h, void* work, double* grad_theta, void* stream);
int lbm_adjoint_get(lbm_handle* h, void* work, double* dst, void* stream);
int lbm_adjoint_set(lbm_handle* h, void* work, const double* src, void* stream);

/*
 * HBM streaming probe (measurement only, no part of the method): streams `bytes`
 * (a multiple of 16; 16-byte aligned device buffers) with non-temporal 16-byte
 * accesses over `grid` work-groups of 256 threads.  mode 0 copies src to dst (one
 * read and one write per byte, the traffic pattern of a step), 1 reads src only (dst
 * must hold 1 KiB; written only for negative input), 2 writes dst only.  Returns
 * LBM_EINVAL for bad arguments.  Asynchronous on `stream`; time it with events.
 */
int lbm_probe_stream(const void* src, void* dst, size_t bytes, int32_t mode, int32_t grid, void* stream);

/* Number of steps taken since lbm_init (host counter). */
int64_t lbm_step_count(const lbm_handle* h);

void lbm_destroy(lbm_handle* h);
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_GP_TERNARY_H */

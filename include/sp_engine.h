/*
 * sp_engine.h -- C ABI of the MI355X atomistic-spin engine.
 *
 * The engine evaluates the effective field of the extended Heisenberg
 * Hamiltonian and advances the Landau-Lifshitz-Gilbert equation with
 * Depondt's rotation-based Heun scheme, following
 * "Spirit: Multifunctional Framework for Atomistic Spin Simulations"
 * (arXiv:1901.11350).  Every compute step runs in hand-written HIP kernels
 * for gfx950.
 *
 * Conventions shared by all calls
 * -------------------------------
 * Units: meV (energies, J, D, K), Tesla (B), Bohr magnetons (mu),
 *        Angstrom (lattice constant), picoseconds (dt), Kelvin (T).
 * Site index: i = a + Na*(b + Nb*(c + Nc*beta)) for cell (a, b, c) and
 *        basis atom beta (each sublattice is a dense Na x Nb x Nc grid).
 * Vector fields are structure-of-arrays: x[N] then y[N] then z[N].
 * Host pointers are always double; device-pointer (_dev) variants use the
 *        engine precision (float for SP_F32, double for SP_F64).
 * Ownership: host arrays are copied in/out before the call returns; _dev
 *        variants borrow caller memory for the call only and are ordered on
 *        the engine stream (no synchronisation with other streams).
 * Errors: every int-returning call returns SP_OK (0) or a negative
 *        sp_status; no C++ exception crosses the ABI.  sp_last_error gives
 *        a message for the last failing call.  A failing set_* call leaves
 *        the previous state unchanged, except when device memory or a HIP
 *        call fails while a new Hamiltonian is installed (SP_E_NOMEM,
 *        SP_E_HIP from sp_set_hamiltonian / sp_set_pairs): the Hamiltonian
 *        and the spins are then dropped and must be set again.
 * Call order: sp_set_geometry -> sp_set_hamiltonian -> sp_set_spins ->
 *        compute calls; out of order gives SP_E_ORDER.
 * Threads: one engine must not be used from two threads at once; separate
 *        engines are independent.
 */
#ifndef SP_ENGINE_H
#define SP_ENGINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sp_engine sp_engine;

enum sp_status {
    SP_OK = 0,
    SP_E_ARG = -1,          /* invalid argument (size, pointer, value) */
    SP_E_ORDER = -2,        /* call made before the state it needs was set */
    SP_E_HIP = -3,          /* HIP runtime error */
    SP_E_NOMEM = -4,        /* device allocation failed */
    SP_E_UNSUPPORTED = -5,  /* valid request this build does not support */
    SP_E_NONFINITE = -6     /* non-finite torque detected during sp_run */
};

enum sp_precision { SP_F32 = 0, SP_F64 = 1 };
enum sp_dmi_kind { SP_DMI_BULK = 1, SP_DMI_INTERFACIAL = 2 };
enum sp_ddi_mode { SP_DDI_OFF = 0, SP_DDI_DIRECT = 1, SP_DDI_SURROGATE = 2, SP_DDI_FFT = 3 };

#define SP_MAX_BASIS 8
#define SP_MAX_SHELLS 8
#define SP_MAX_GAUSS 16

/* Hamiltonian parameters (Sec. III.A, extended Heisenberg Hamiltonian):
 *   H = - sum_i mu_i mu_B B . n_i - sum_i K_i (K_hat_i . n_i)^2
 *       - sum_<ij> J_ij n_i . n_j - sum_<ij> D_ij . (n_i x n_j)
 *       + 1/2 C_dd sum_{i != j} mu_i mu_j [n_i.n_j - 3 (n_i.r_ij)(n_j.r_ij)] / r_ij^3
 * over unique pairs <ij>.  J and D are given per neighbour shell (shell s =
 * the s-th distinct neighbour distance of a basis atom).  The scalar D of a
 * shell becomes the vector D r_hat_ij (bulk) or D (z x r_hat_ij)
 * (interfacial).  The dipole term is summed over the sites of the sample
 * (no periodic images).  mu, K, K_axis are per basis atom. */
typedef struct {
    int n_basis;             /* must equal the geometry's n_basis */
    const double *mu;        /* [n_basis], Bohr magnetons, > 0 */
    double B[3];             /* Tesla */
    const double *K;         /* [n_basis], meV (may be NULL: all zero) */
    const double *K_axis;    /* [3*n_basis], normalised internally (may be NULL if K is) */
    int n_exch_shells;       /* 0..SP_MAX_SHELLS */
    const double *J;         /* [n_exch_shells], meV */
    int n_dmi_shells;        /* 0..SP_MAX_SHELLS */
    const double *D;         /* [n_dmi_shells], meV */
    int dmi_kind;            /* SP_DMI_BULK or SP_DMI_INTERFACIAL */
    int ddi_mode;            /* SP_DDI_OFF, SP_DDI_DIRECT, SP_DDI_SURROGATE (learned
                                field with residual check and direct-sum fallback,
                                see sp_ddi_*), or SP_DDI_FFT: the same pair sum
                                (all pairs inside the sample, Sec. III.A) as a 2D
                                convolution per plane pair, zero-padded FFTs along
                                a and b; needs n_cells[0], n_cells[1] <= 512 and
                                n_cells[2] * n_basis <= 64, else
                                SP_E_UNSUPPORTED from sp_set_hamiltonian */
    int n_gauss;             /* 0..SP_MAX_GAUSS on-site Gaussian potentials, the same on
                                every site: sum_k a_k exp(-(1 - n.c_k)^2 / (2 sigma_k^2))
                                (the single-spin landscape of Appendix G; c_k are
                                normalised internally; reported with the anisotropy
                                energy; runs on the two-pass step path) */
    const double *gauss_a;       /* [n_gauss], meV */
    const double *gauss_sigma;   /* [n_gauss], > 0 */
    const double *gauss_c;       /* [3*n_gauss], non-zero centre vectors */
} sp_hamiltonian;

/* Integrators of dn/dt = n x A (Sec. III.C):
 * SP_SOLVER_DEPONDT  Depondt's rotation form of Heun's scheme (Appendix B):
 *                    n^p = R(A(n)) n, n' = R((A(n) + A(n^p))/2) n;
 * SP_SOLVER_HEUN     Heun's method (Appendix B): n^p = n + dt n x A(n) and
 *                    n' = n + dt (n x A(n) + n^p x A(n^p))/2, both stages
 *                    renormalised;
 * SP_SOLVER_SIB      the semi-implicit midpoint scheme B (Appendix C): each
 *                    stage solves x = n + dt (n + x)/2 x A with A frozen,
 *                    first at n, then at the midpoint (n + n^p)/2.
 * All three use the same thermal normals in both stages. */
enum sp_solver { SP_SOLVER_DEPONDT = 0, SP_SOLVER_HEUN = 1, SP_SOLVER_SIB = 2 };

/* LLG parameters (Sec. III.C).  T > 0 adds the stochastic thermal field
 * sqrt(2 alpha k_B T / (gamma mu_i mu_B dt)) eta_i, eta_i three standard
 * normals per site and step from Philox4x32-10 with counter
 * (site, step_lo, step_hi, replica) and key (seed_lo, seed_hi), via
 * u = (x + 1/2) 2^-32 and Box-Muller on (u0,u1), (u2,u3). */
typedef struct {
    double alpha;            /* Gilbert damping, >= 0 */
    double dt_ps;            /* time step, > 0 */
    double T_K;              /* temperature, >= 0 */
    uint64_t seed;           /* Philox key */
    uint32_t replica;        /* Philox counter word 3 (replica index) */
    int32_t solver;          /* sp_solver; replica batches take SP_SOLVER_DEPONDT only */
} sp_llg_params;

/* Observables of one spin state.  per_term: Zeeman, anisotropy, exchange,
 * DMI, dipole (meV).  max_torque = max_i |n_i x dH/dn_i| (meV); M = mean
 * spin (1/N) sum_i n_i; max_norm_dev = max_i | |n_i| - 1 |.  All reduced in
 * double precision. */
typedef struct {
    int64_t step;
    double E;
    double per_term[5];
    double max_torque;
    double M[3];
    double max_norm_dev;
} sp_observation;

/* Metropolis Monte Carlo parameters (Sec. III.B). */
typedef struct {
    double T_K;              /* temperature, > 0 */
    double cone_deg;         /* opening angle of the trial cone, (0, 180] degrees (initial, if adaptive) */
    uint64_t seed;           /* Philox key */
    uint32_t replica;        /* Philox counter word 3 */
    double target_acceptance;/* 0: fixed cone; in (0, 1): the cone follows the acceptance feedback */
} sp_mc_params;

/* Create an engine on HIP device `device` computing in `precision`.
 * hip_stream: a hipStream_t to order all work on, or NULL for an engine-owned
 * stream.  *out receives the engine (NULL on failure). */
int sp_create(sp_engine **out, int device, int precision, void *hip_stream);
/* Free the engine and all device memory it owns.  NULL is ignored. */
void sp_destroy(sp_engine *e);
/* Message of the last failing call on this engine (never NULL). */
const char *sp_last_error(const sp_engine *e);

/* Metropolis sweeps with cone trial moves (Sec. III.B).  The paper's sweep
 * picks every spin once, sequentially in random order; here a sweep tries
 * every site once, colour after colour, with a periodic colouring of the
 * sites -- site (a, b, c, beta) takes the colour of its class
 * (a mod ma, b mod mb, c mod mc, beta), periods 1-6 per axis dividing the
 * length of each periodic axis, classes coloured by DSATUR on the quotient
 * graph of the bonds, fewest colours chosen -- so that no bond joins two
 * sites of one colour (the checkerboard for the simple-cubic nearest-
 * neighbour lattice): a colour updates in parallel and every trial sees the
 * current state of its neighbours; the same Boltzmann distribution,
 * sampled by another schedule.
 * Trial at site i of sweep s: Philox block of counter (i, s_lo, s_hi,
 * replica) and key (seed_lo, seed_hi), u_k = (x_k + 1/2) 2^-32; phi = 2 pi u0,
 * cos(theta) = 1 - u1 (1 - cos(cone)); new spin cos(theta) n +
 * sin(theta) (cos(phi) e1 + sin(phi) e2), e1 = unit(n x r) with r = z if
 * |n_z| < 0.9 else x, e2 = n x e1; accepted if u2 < exp(-dE / (k_B T)).
 * Trial, dE and the test are computed in FP64 in both engine precisions
 * (an FP32 engine reads its FP32 spins and stores an accepted trial rounded
 * to FP32).  The sweep number is the engine's step counter (advanced by
 * n_sweeps).  Adaptive cone (target_acceptance > 0; the paper's feedback
 * toward a desired acceptance ratio, whose rule it does not print): after
 * every sweep with acceptance ratio a the cone is multiplied by
 * 1 + a - target_acceptance, at most 180 degrees, on the device; *cone_out
 * (may be NULL) receives the cone after the last sweep.
 * Any basis; needs no dipole term and a colouring within those periods
 * (SP_E_UNSUPPORTED otherwise, e.g. a periodic axis too short for its
 * bonds).  obs
 * receives n_sweeps / observe_every observations (observe_every = 0: none);
 * *accepted (may be NULL) the accepted trials of the run. */
int sp_mc_run(sp_engine *e, const sp_mc_params *p, int64_t n_sweeps, int64_t observe_every,
              sp_observation *obs, int64_t *accepted, double *cone_out);
/* Version string of the library. */
const char *sp_version(void);

/* Geometry: Bravais lattice with basis (Sec. III.A; arbitrary Bravais vectors
 * and basis cells).  bravais: rows a1, a2, a3 in units of the lattice
 * constant; basis: n_basis cartesian positions in the same units;
 * n_cells[k] >= 1; periodic[k] in {0, 1}; lattice_constant in Angstrom.
 * Invalidates the Hamiltonian and spins. */
int sp_set_geometry(sp_engine *e, const double bravais[9], int n_basis, const double *basis,
                    const int n_cells[3], const int periodic[3], double lattice_constant);
/* Hamiltonian; builds the neighbour-shell bond table.  Requires geometry.
 * SP_E_ARG if a requested shell does not exist within 4 cells. */
int sp_set_hamiltonian(sp_engine *e, const sp_hamiltonian *h);

/* Explicit pair interactions.  The exchange and DMI sums of the Hamiltonian
 * (Sec. III.A, the extended Heisenberg Hamiltonian) run over unique pairs
 * <ij>, with no limit on their number, distance or direction dependence.  Pair p couples basis atom
 * bi[p] of every cell x with basis atom bj[p] of cell x + dcell[3p..3p+2]
 * (cell offsets along a1, a2, a3) with energy
 *   -J[p] n_i.n_j - D_p.(n_i x n_j),   D_p = D[3p..3p+2] in meV (D may be NULL).
 * Periodic axes wrap the partner (also by more than one lattice length),
 * open axes drop the pair where the partner leaves the lattice, and a pair
 * that wraps onto its own site is dropped.  Replaces the shell-built
 * exchange and DMI bonds of the current Hamiltonian (call after
 * sp_set_hamiltonian, which discards the pairs again); every other term
 * stays, spins are kept, and the step path is chosen again (the
 * compile-time-stencil paths shape2d/shape3d/persist2d are not used with
 * explicit pairs).  n_pairs = 0 removes exchange and DMI.  SP_E_ARG for: a
 * pair given twice or together with its reverse (bj, bi, -dcell), a spin
 * paired with itself (bi == bj, dcell = 0), basis indices out of range,
 * |dcell| > 64 on an axis, non-finite J or D, or more than 256 bonds on
 * one basis atom (both directions of every pair counted).  Arrays are read
 * during the call only. */
int sp_set_pairs(sp_engine *e, int64_t n_pairs, const int *bi, const int *bj, const int *dcell,
                 const double *J, const double *D);
/* Number of sites N (0 before sp_set_geometry). */
int64_t sp_num_sites(const sp_engine *e);
/* Directed bonds of basis atom beta in the bond table (bonds whose J and D
 * are both zero are omitted): out[10*k .. 10*k+9] =
 * (beta_j, da, db, dc, shell, J, Dx, Dy, Dz, 0) as doubles for the first
 * max_bonds bonds (out may be NULL).  Returns the bond count or a negative
 * status. */
int sp_get_bonds(sp_engine *e, int beta, double *out, int max_bonds);

/* Spins: n_soa holds 3N doubles; every vector is normalised on input; a
 * zero-length or non-finite vector gives SP_E_ARG.  Resets nothing else. */
int sp_set_spins(sp_engine *e, const double *n_soa, int64_t N);
int sp_get_spins(sp_engine *e, double *n_soa, int64_t N);
/* Device-side variants in engine precision (no normalisation on set). */
int sp_set_spins_dev(sp_engine *e, const void *n_soa_dev, int64_t N);
int sp_get_spins_dev(sp_engine *e, void *n_soa_dev, int64_t N);

/* Step counter (the Philox counter of the next step). */
int sp_set_step(sp_engine *e, uint64_t step);
uint64_t sp_get_step(const sp_engine *e);

/* Gradient dH/dn_i in the embedding space (meV), all terms of the extended
 * Heisenberg Hamiltonian of Sec. III.A (Zeeman, anisotropy, exchange, DMI,
 * dipole, on-site Gaussians); the effective field of Sec. III.C is
 * B_eff = -g (divide by mu_i mu_B for Tesla).  g_soa: 3N doubles written
 * before return.  SP_E_ORDER before sp_set_spins; SP_E_ARG if N is not the
 * engine's site count.  sp_gradient_dev writes 3N values of the engine precision to device memory
 * on the engine's stream; on FP32 lattices with a compile-time stencil whose
 * sides divide into 64 x 64 tiles (at least 512 of them) a 16-byte aligned
 * g_soa_dev takes the 16-byte load/store kernel (same values, bit for bit). */
int sp_gradient(sp_engine *e, double *g_soa, int64_t N);
int sp_gradient_dev(sp_engine *e, void *g_soa_dev, int64_t N);
/* Energy of the current state, total and by term (Zeeman, anisotropy,
 * exchange, DMI, dipole; meV), the Hamiltonian of Sec. III.A evaluated as
 * E = sum_i n_i.(g_lin + g_quad / 2) with the linear (Zeeman) and quadratic
 * parts of the gradient (Appendix H), reduced in double precision in a
 * fixed order.  per_term may be NULL.  SP_E_ORDER before sp_set_spins. */
int sp_energy(sp_engine *e, double *E_total, double per_term[5]);
/* All observables of the current state (sp_observation): the energies of
 * sp_energy, the maximum torque max_i |n_i x dH/dn_i| (the quantity a
 * minimiser drives to zero: damping-only LLG of Sec. III.C and the
 * velocity projection of Appendix D), the mean spin and the largest
 * deviation of |n_i| from one.  *obs is written before return. */
int sp_observe(sp_engine *e, sp_observation *obs);

/* One Depondt step (Appendix B): predictor n^p = R(A(n)) n, corrector
 * n(t+dt) = R((A(n) + A(n^p))/2) n with the same thermal normals in both.
 * Advances the step counter by one. */
int sp_llg_step(sp_engine *e, const sp_llg_params *p);
/* n_steps steps of the LLG equation of Sec. III.C with the solver of p
 * (Depondt by default, Appendix B), the thermal field drawn per step and
 * site from the Philox stream.  If observe_every > 0 an observation is
 * taken after every observe_every steps and written to obs[k] (obs must
 * hold n_steps/observe_every entries; may be NULL to only check
 * finiteness).  When an observation finds a non-finite torque the remaining
 * steps are skipped and SP_E_NONFINITE is returned (sp_last_error names the
 * step).  Chunks of observe_every steps (32 without observations) are
 * captured once as HIP graphs and replayed while parameters, buffers and
 * step path stay the same (sp_set_graph_replay turns this off); results are
 * the same bit for bit either way. */
int sp_run(sp_engine *e, const sp_llg_params *p, int64_t n_steps, int64_t observe_every,
           sp_observation *obs);
/* sp_run with the convergence test of a relaxation (damping-only LLG as a
 * minimiser, Sec. III.C; the paper prints no criterion): the run stops after
 * the first observation whose maximum torque max_i |n_i x dH/dn_i| (FP64
 * reduction) is below tol, or after max_steps steps.  The test runs on the
 * device (no host synchronisation per observation); the state and the step
 * counter are those of the observation that passed.  observe_every > 0 and
 * tol > 0 (SP_E_ARG otherwise).  obs (may be NULL) receives the
 * observations taken, up to max_steps/observe_every entries;
 * *steps_done (may be NULL) the steps taken.  SP_E_NONFINITE as sp_run. */
int sp_run_tol(sp_engine *e, const sp_llg_params *p, int64_t max_steps, int64_t observe_every, double tol,
               sp_observation *obs, int64_t *steps_done);
/* Graph replay of sp_run on (enable != 0, the default) or off (direct
 * launches; cached graphs are freed). */
int sp_set_graph_replay(sp_engine *e, int enable);
/* Wait for all work queued on the engine stream. */
int sp_synchronize(sp_engine *e);

/* Dipole-dipole gradient alone: the dipolar term of the Hamiltonian of
 * Sec. III.A (in the physical form 1/2 C_dd sum_{i!=j} mu_i mu_j
 * [n_i.n_j - 3 (n_i.r)(n_j.r)] / r^3) over all pairs of the sample (open,
 * no periodic images), evaluated as ddi_mode says: the direct sum
 * (SP_DDI_DIRECT), the FFT convolution of the same sum (SP_DDI_FFT) or the
 * learned field with its residual check (SP_DDI_SURROGATE).  g_soa
 * receives 3N doubles (meV).  sp_dipole_gradient_dev reads n_soa_dev and
 * writes g_soa_dev (engine precision, 3N each, caller-owned device memory,
 * engine stream).  SP_E_ORDER when ddi_mode is off. */
int sp_dipole_gradient(sp_engine *e, double *g_soa, int64_t N);
int sp_dipole_gradient_dev(sp_engine *e, const void *n_soa_dev, void *g_soa_dev, int64_t N);
/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The direct
 * sum of sp_dipole_gradient_dev (whatever ddi_mode, which must not be off)
 * with its partial sums in a file-scope device array of 32 MiB per GPU
 * instead of engine memory; it calls no allocating routine.  The caller
 * passes inputs and outputs as for sp_dipole_gradient_dev (same values, bit
 * for bit, as its SP_DDI_DIRECT result).  SP_E_ARG when the partial sums
 * (3 N x slices values of the engine precision; slices = 16 up to 65,536
 * sites, then about 2^20 / N) exceed 32 MiB, e.g. beyond about 1.4 M sites
 * in FP64 or 2.8 M in FP32.  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (engines on different streams) race and
 * must be ordered by the caller. */
int sp_dipole_gradient_dev_noalloc(sp_engine *e, const void *n_soa_dev, void *g_soa_dev, int64_t N);

/* The three independent standard normals per site and step of the
 * stochastic field of Sec. III.C, exactly as the LLG kernels draw them:
 * Philox4x32-10 block of counter (site, step_lo, step_hi, replica) and key
 * (seed_lo, seed_hi), u_k = (x_k + 1/2) 2^-32, Box-Muller on (u0, u1) and
 * (u2, u3), first three normals; for n_sites consecutive sites starting at
 * site0.  eta_soa receives 3*n_sites values (engine precision, as double,
 * SoA); raw4 (may be NULL) the 4*n_sites Philox words.  For tests of the
 * generator. */
int sp_thermal_normals(sp_engine *e, uint64_t seed, uint64_t step, uint32_t replica,
                       uint32_t site0, int64_t n_sites, double *eta_soa, uint32_t *raw4);

/* Name of the kernel path sp_llg_step uses for the current state
 * ("fused2d", "twopass", ...), for diagnostics. */
const char *sp_step_path(const sp_engine *e);
/* Force the step path: "twopass" (any lattice), "fused2d" (one-atom 2D
 * lattice, runtime bond loop), "fusedtile" (lattice with a basis -- 2D with
 * 2-4 atoms and bond reach <= 2, 3D with 1-3 atoms, FP64 1-2, reach 1 --
 * or a 3D one-atom lattice without a compile-time stencil; no dipole or
 * Gaussian terms; LDS tiles of every atom, runtime bond table; also the
 * path of sp_gradient on such lattices), "shape2d[/TXxTYxNT]" (one-atom 2D lattice
 * whose bond table matches a compile-time stencil; optional tile
 * configuration such as "shape2d/32x16x256"), "shape3d[/cfg]" (one-atom
 * simple-cubic lattice with a compile-time stencil) or "persist2d[/TXxTY]"
 * (as shape2d; tiles "64x16", "32x32", "32x16" in FP32, "32x16" in FP64;
 * lattice sides must be multiples of the tile and every tile must fit on
 * the device at once).  On persist2d, sp_run advances the Depondt solver
 * many steps per launch (one launch per observation interval): tiles stay
 * resident and exchange halos through per-tile flags with agent-scope
 * release/acquire; a tile that waits for its neighbours beyond a bound
 * (about a second; environment variable SP_PERSIST_SPIN_LIMIT lowers it)
 * makes sp_run return SP_E_HIP with the spins invalid.  sp_llg_step and the
 * other solvers use the one-step kernel of the same tile on that path.
 * A path the current lattice does not allow gives SP_E_UNSUPPORTED, an
 * unknown name SP_E_ARG.  Reset by sp_set_hamiltonian (which picks the
 * default path of the lattice). */
int sp_set_step_path(sp_engine *e, const char *name);
/* Autotuner: times every step path and tile configuration the current
 * lattice allows (n_steps steps each, after one warm-up step, HIP events on
 * the engine stream) from the current spins, then keeps the fastest.  Spins
 * and the step counter are restored.  *ms_per_step (may be NULL) receives the
 * best time per step. */
int sp_autotune(sp_engine *e, const sp_llg_params *p, int n_steps, double *ms_per_step);

/* ------------------------------------------------------------------------
 * Replica batches.  Many independent systems that share one Hamiltonian but
 * differ in size, temperature, damping, time step and Philox replica index
 * advance together: replicas small enough for one workgroup's LDS (32x32 and
 * 64x64) stay resident in LDS for a whole chunk of steps; larger ones run as
 * (replica, tile) work items of one launch per step.  A chunk of K steps is
 * captured once as a HIP graph (resident branch in parallel with the K tiled
 * launches) and replayed; the step number lives in device memory.  Small
 * systems are otherwise bound by launch overhead, which the paper notes for
 * its GPU back end at small sizes (Sec. II).  FP32 only.
 * ------------------------------------------------------------------------ */
typedef struct sp_batch sp_batch;

int sp_batch_create(sp_batch **out, int device, void *hip_stream);
void sp_batch_destroy(sp_batch *b);
const char *sp_batch_last_error(const sp_batch *b);
/* Add a replica taking geometry, Hamiltonian and current spins from engine e
 * (FP32, one-atom 2D lattice whose bond table matches a compile-time
 * stencil, spins set) and LLG parameters p (p->replica is its Philox replica
 * index).  Every replica must have the same Hamiltonian.  The batch copies
 * what it needs; e may be destroyed afterwards.  Returns the slot (>= 0) or a
 * negative status.  No replica can be added after the first sp_batch_run. */
int sp_batch_add(sp_batch *b, sp_engine *e, const sp_llg_params *p);
/* Advance every replica by n_steps Depondt steps. */
int sp_batch_run(sp_batch *b, int64_t n_steps);
/* Spins of one replica (3N doubles, SoA). */
int sp_batch_get_spins(sp_batch *b, int slot, double *n_soa, int64_t N);
/* Size of one replica and whether it runs LDS-resident (1) or tiled (0). */
int sp_batch_replica_info(sp_batch *b, int slot, int64_t *n_sites, int *resident);
/* Graph chunk length in steps (even, 2..1024; default 32). */
int sp_batch_set_chunk(sp_batch *b, int steps);
/* Step number of the next batch step (shared by all replicas). */
uint64_t sp_batch_get_step(const sp_batch *b);
/* Times each tile configuration of the tiled kernel for n_steps steps,
 * keeps the fastest, restores all replicas.  *ms_per_step may be NULL. */
int sp_batch_autotune(sp_batch *b, int n_steps, double *ms_per_step);

typedef struct sp_gneb sp_gneb;
/* Attach a GNEB chain (sp_gneb_create, below; FP32 engine, same device) to
 * the batch: every sp_batch_run(b, n) then also performs n velocity-
 * projection iterations of the chain (Sec. III.D), on a branch of the same
 * chunk graph that runs beside the replicas, with the same kernels and
 * results as sp_gneb_iterate(g, n).  While attached, sp_gneb_iterate on the
 * chain returns SP_E_ORDER and the chain's readers (sp_gneb_get_chain,
 * sp_gneb_get_forces, sp_gneb_set_image_type) wait for the batch's work.
 * Destroying either object detaches the chain (it stays usable on its own).
 * SP_E_ORDER if the batch already has a chain or the chain another batch;
 * SP_E_ARG for an FP64 chain or another device.  sp_batch_autotune times
 * the replicas only and leaves an attached chain as it is. */
int sp_batch_add_gneb(sp_batch *b, sp_gneb *g);

/* ------------------------------------------------------------------------
 * Geodesic nudged elastic band (Sec. III.D; Appendix F for the tangents,
 * geodesic distances and per-spin projections; Appendix D for the
 * velocity-projection minimiser).  Per interior image v the force is
 *   F = -g + (g.t)t (then projected per spin onto the tangent plane)
 *       + k (l_{v,v+1} - l_{v-1,v}) t,
 * t the improved tangent (difference towards the higher-energy neighbour,
 * energy-weighted at extrema), projected per spin and normalised in 3N;
 * l the geodesic distance sqrt(sum_i angle(n_i, n'_i)^2).  Images 0 and M-1
 * stay fixed.  The velocity projection runs chain-wide: Verlet steps of
 * mass vp_mass and step vp_dt, v <- (v.F/|F|^2) F when v.F > 0 else 0, spins
 * renormalised after each move.  Energies and all dot products are reduced
 * in double precision.
 * ------------------------------------------------------------------------ */

/* Chain of n_images (>= 3) images on engine e's lattice and Hamiltonian (no
 * dipole term), in e's precision.  chain: n_images*3N doubles, image-major,
 * each image SoA; spins are normalised on input.  The chain borrows e: e
 * must outlive it and keep its geometry and Hamiltonian. */
int sp_gneb_create(sp_gneb **out, sp_engine *e, int n_images, const double *chain, double k_spring,
                   double vp_dt, double vp_mass);
void sp_gneb_destroy(sp_gneb *c);
const char *sp_gneb_last_error(const sp_gneb *c);
/* Image types (Sec. III.D): SP_IMAGE_CLIMBING drops the spring force and
 * inverts the energy gradient along the path (F = -grad E + 2 (grad E . tau)
 * tau); SP_IMAGE_FALLING drops the spring force and keeps the full energy
 * force (F = -grad E), so the image relaxes into a minimum; both per-spin
 * projected.  image in 1..n_images-2; SP_E_ARG otherwise.  Takes effect at
 * the next iteration (the minimiser's previous force is kept). */
enum sp_image_type { SP_IMAGE_NORMAL = 0, SP_IMAGE_CLIMBING = 1, SP_IMAGE_FALLING = 2 };
int sp_gneb_set_image_type(sp_gneb *c, int image, int type);
/* n_iter velocity-projection iterations. */
int sp_gneb_iterate(sp_gneb *c, int n_iter);
/* Relaxation of the chain to its minimum energy path: velocity-projection
 * iterations (Appendix D) with the chain's GNEB forces (Sec. III.D) until the
 * largest per-spin force |F_{v,i}| of the interior images (FP64 maximum) is
 * below tol, or max_iter iterations.  The test runs on the device after
 * every iteration; once it passes the remaining launches return at once, so
 * the chain is that of the iteration that passed (as after
 * sp_gneb_iterate(c, *iters_done)).  tol > 0 and max_iter >= 0 (SP_E_ARG
 * otherwise); SP_E_ORDER while attached to a batch.  *iters_done (may be
 * NULL) receives the iterations taken. */
int sp_gneb_iterate_tol(sp_gneb *c, int max_iter, double tol, int *iters_done);
/* Current chain (n_images*3N doubles). */
int sp_gneb_get_chain(sp_gneb *c, double *chain);
/* Of the last force evaluation: image energies E[n_images], geodesic
 * distances l[n_images-1], forces F[n_images*3N] (any may be NULL). */
int sp_gneb_get_forces(sp_gneb *c, double *E, double *l, double *F);

/* ------------------------------------------------------------------------
 * Learned dipole field (not in the paper; a stand-in for its costliest term,
 * the dipolar direct sum of Sec. III.A).  A stack of zero-padded 3x3
 * convolutions with SiLU between layers maps the spins of a one-atom film
 * (channels 3 x number of layers, c = 3*layer + component, pixels = the
 * in-plane cells) to the dipole gradient divided by C_dd mu^2.  Matrix-core
 * kernels: bf16 operands, FP32 accumulation (v_mfma_f32_16x16x32_bf16),
 * trained by the library's own forward/backward kernels and Adam on FP32
 * master weights.  With ddi_mode SP_DDI_SURROGATE every dipole evaluation of
 * the LLG step uses the network, then computes the exact direct sum at
 * n_check sampled sites; when the relative error there exceeds tol the full
 * direct sum replaces the network's field (decided on the device).
 * Requirements: FP32 engine, n_basis 1, Na and Nb multiples of 16,
 * 3*Nc <= 32, a Hamiltonian with a dipole term (any ddi_mode but OFF).
 * Device arrays hold `batch` samples of 3N floats each (SoA per sample).
 * ------------------------------------------------------------------------ */
/* (Re)create the network: channels[0..n_layers] with channels[0] and
 * channels[n_layers] = 3*Nc, each <= 32; He-normal weights from seed. */
int sp_ddi_init(sp_engine *e, int n_layers, const int *channels, uint64_t seed);
/* Residual form of the learned field (the other sp_ddi_* calls then act on
 * it): the film is cut into blocks of block x block cells and every layer
 * (block^2 x layers = 64 sites); the backbone sums the sites of the blocks
 * within `reach` (0..2) blocks of a site's block exactly and every other
 * block as one dipole (its moment at its centroid); the network (12 input
 * channels: the block's moment and first moments; 12 output channels: the
 * coefficients c0, c1 of a correction c0 + (r_i - R_b) . c1 per block) runs
 * on the block grid and is trained on the least-squares fit of (direct sum
 * - backbone) per block.  The field is scale x (backbone + correction).
 * Needs an FP32 engine on a one-atom simple-cubic film whose sides are
 * multiples of 16 blocks, channels[0] = channels[n_layers] = 12
 * (SP_E_UNSUPPORTED / SP_E_ARG otherwise).  Replaces any previous network. */
int sp_ddi_init_residual(sp_engine *e, int n_layers, const int *channels, uint64_t seed, int block, int reach);
/* Residual form: the backbone field alone (the method without the network),
 * batch samples, layout as sp_ddi_forward_dev. */
int sp_ddi_backbone_dev(sp_engine *e, int batch, const void *spins_dev, void *field_dev);
/* Parameter count and host copies (per layer: w[ky][kx][ci][co] then b[co]). */
int64_t sp_ddi_num_params(sp_engine *e);
int sp_ddi_set_params(sp_engine *e, const double *params, int64_t n);
int sp_ddi_get_params(sp_engine *e, double *params, int64_t n);
/* Training labels: the direct-sum dipole gradient (meV) of each sample. */
int sp_ddi_label_dev(sp_engine *e, int batch, const void *spins_dev, void *labels_dev);
/* Network field (meV) of each sample. */
int sp_ddi_forward_dev(sp_engine *e, int batch, const void *spins_dev, void *field_dev);
/* Loss sum_b |net_b - labels_b/(C_dd mu^2)|^2 / |labels_b/(C_dd mu^2)|^2 and
 * its gradient (host, parameter layout; may be NULL). */
int sp_ddi_loss_grad_dev(sp_engine *e, int batch, const void *spins_dev, const void *labels_dev, double *loss,
                         double *grad);
/* Adam (lr, beta 0.9/0.999, eps 1e-8) over `epochs` shuffled passes of
 * minibatches of `batch` samples; epoch_loss[epochs] (may be NULL) receives
 * the mean loss per sample of each epoch. */
int sp_ddi_train_dev(sp_engine *e, int n_samples, const void *spins_dev, const void *labels_dev, int epochs,
                     int batch, double lr, uint64_t seed, double *epoch_loss);
/* Residual check: tolerance on the sampled relative error, number of
 * sampled sites (0..4096; 0 disables check and fallback). Default 1e-3, 256. */
int sp_ddi_configure(sp_engine *e, double tol, int n_check_sites);
/* out[4] = evaluations, fallbacks, last sampled error, max sampled error. */
int sp_ddi_stats(sp_engine *e, double out[4]);

#ifdef __cplusplus
}
#endif
#endif

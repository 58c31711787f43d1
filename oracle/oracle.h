/*
 * oracle.h -- plain FP64 CPU oracle for the atomistic spin hot path of
 * "Spirit: Multifunctional Framework for Atomistic Spin Simulations"
 * (arXiv:1901.11350).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source,
 * header, table or helper with the HIP engine; both only receive the same
 * seeded input arrays.
 *
 * Everything is double precision, scalar loops, no FMA contraction
 * (built with -ffp-contract=off), optional OpenMP over sites.
 *
 * Units: meV, Tesla, Bohr magneton, Angstrom, picosecond, Kelvin.
 * Spin / field arrays are structure-of-arrays: x[N], y[N], z[N] stored
 * contiguously (3N doubles), site index i = a + Na*(b + Nb*(c + Nc*beta)).
 */
#ifndef SPIN_ORACLE_H
#define SPIN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_MAX_BASIS 8
#define ORA_MAX_SHELLS 8
#define ORA_MAX_BONDS_PER_BASIS 256

enum { ORA_DMI_BULK = 1, ORA_DMI_INTERFACIAL = 2 };
#define ORA_MAX_GAUSS 16

typedef struct {
    double bravais[9];                 /* rows a1, a2, a3 (units of the lattice constant) */
    int n_basis;
    double basis[3 * ORA_MAX_BASIS];   /* cartesian, units of the lattice constant */
    int n_cells[3];
    int periodic[3];
    double lattice_constant;           /* Angstrom */
} ora_geometry;

typedef struct {
    double mu[ORA_MAX_BASIS];          /* Bohr magnetons per basis atom */
    double B[3];                       /* Tesla */
    double K[ORA_MAX_BASIS];           /* meV per basis atom */
    double K_axis[3 * ORA_MAX_BASIS];  /* unit axes per basis atom */
    int n_exch;
    double J[ORA_MAX_SHELLS];          /* meV per shell */
    int n_dmi;
    double D[ORA_MAX_SHELLS];          /* meV per shell */
    int dmi_kind;                      /* ORA_DMI_BULK or ORA_DMI_INTERFACIAL */
    int ddi;                           /* 1: include dipole-dipole direct sum */
    /* on-site Gaussian potentials sum_k a_k exp(-(1 - n.c_k)^2 / (2 sigma_k^2))
     * on every site (the single-spin landscape of Appendix G); c_k are
     * normalised internally; reported with the anisotropy energy */
    int n_gauss;
    double gauss_a[ORA_MAX_GAUSS];     /* meV */
    double gauss_sigma[ORA_MAX_GAUSS];
    double gauss_c[3 * ORA_MAX_GAUSS];
} ora_hamiltonian;

/* One directed bond of a basis atom: from basis atom `bi` in cell x to basis
 * atom `bj` in cell x + (da, db, dc). */
typedef struct {
    int bi, bj, da, db, dc, shell;
    double J;
    double D[3];
} ora_bond;

typedef struct ora_system ora_system;

ora_system *ora_create(const ora_geometry *g, const ora_hamiltonian *h);
void ora_destroy(ora_system *s);
int64_t ora_num_sites(const ora_system *s);

/* Bond table (per basis atom, both directions kept).  Returns the number of
 * bonds written (at most max_bonds). */
int ora_bonds(const ora_system *s, ora_bond *out, int max_bonds);
/* Explicit neighbour list of one site: returns its degree, fills j / bond ids. */
int ora_site_neighbours(const ora_system *s, int64_t i, int64_t *j_out, int *bond_out, int max_out);
/* Shell distances of basis atom beta (units of the lattice constant). */
int ora_shell_distances(const ora_system *s, int beta, double *out, int max_out);
/* Replace the shell-built exchange/DMI bonds by n explicit unique pairs:
 * pair p joins basis atom bi[p] of every cell x with basis atom bj[p] of
 * cell x + dcell[3p..3p+2], energy -J[p] n_i.n_j - D_p.(n_i x n_j) (D may
 * be NULL).  Returns 0; -1 for an index out of range, a spin paired with
 * itself, a pair given twice or with its reverse, or too many bonds. */
int ora_set_pairs(ora_system *s, int n, const int *bi, const int *bj, const int *dcell, const double *J,
                  const double *D);

/* dH/dn per site (embedding space).  terms, if non-NULL, receives the five
 * contributions Zeeman, anisotropy, exchange, DMI, dipole as 5 blocks of 3N. */
void ora_gradient(const ora_system *s, const double *n, double *g, double *terms);
/* Dipole gradient at a subset of sites only (rows of 3 per requested site). */
void ora_dipole_gradient_sites(const ora_system *s, const double *n, const int64_t *sites,
                               int64_t n_req, double *g_out /* 3*n_req, xyz per site */);
/* Energy by the definition of the Hamiltonian; per_term (may be NULL) gets
 * Zeeman, anisotropy, exchange, DMI, dipole. */
double ora_energy(const ora_system *s, const double *n, double *per_term);

/* Philox4x32-10 block (Salmon, Moraes, Dror, Shaw, SC'11). */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Three standard normals of site `site` at step `step` of replica `replica`:
 * counter (site, step_lo, step_hi, replica), key (seed_lo, seed_hi). */
void ora_thermal_normals(uint64_t seed, uint64_t step, uint32_t site, uint32_t replica,
                         double eta[3]);

enum { ORA_SOLVER_DEPONDT = 0, ORA_SOLVER_HEUN = 1, ORA_SOLVER_SIB = 2 };

typedef struct {
    double alpha;
    double dt;       /* ps */
    double T;        /* K */
    uint64_t seed;
    uint32_t replica;
    int32_t solver;  /* ORA_SOLVER_* */
} ora_llg_params;

/* One Depondt step at step counter `step` (used as the Philox counter). n is
 * updated in place. */
void ora_depondt_step(const ora_system *s, double *n, const ora_llg_params *p, uint64_t step);
/* One step of Heun's method with renormalisation (Appendix B, first part). */
void ora_heun_step(const ora_system *s, double *n, const ora_llg_params *p, uint64_t step);
/* One step of the semi-implicit midpoint scheme SIB (Appendix C). */
void ora_sib_step(const ora_system *s, double *n, const ora_llg_params *p, uint64_t step);
/* One step of the solver p->solver. */
void ora_llg_step(const ora_system *s, double *n, const ora_llg_params *p, uint64_t step);
/* Rotation of one vector about omega by |omega|*dt (exposed for tests). */
void ora_rotate(const double n[3], const double omega[3], double dt, double out[3]);

typedef struct {
    int64_t step;
    double E;
    double per_term[5];
    double max_torque;
    double M[3];
    double max_norm_dev;
} ora_observation;

void ora_observe(const ora_system *s, const double *n, int64_t step, ora_observation *obs);
/* n_steps steps of p->solver starting at step counter step0; an observation is
 * recorded after every observe_every steps (if > 0).  Returns the number of
 * observations written. */
int64_t ora_run(const ora_system *s, double *n, const ora_llg_params *p, uint64_t step0,
                int64_t n_steps, int64_t observe_every, ora_observation *obs);

/* ----------------------------------------------------------- Monte Carlo
 * Metropolis sampling with cone trial moves (Sec. III.B).  One sweep picks
 * every site once, sequentially, in an order drawn at random per sweep
 * (ora_mc_order), and gives it a trial step; no dipole term.
 * Trial at site i of sweep s: Philox block x of counter (i, s_lo, s_hi,
 * replica), key (seed_lo, seed_hi), u_k = (x_k + 1/2) 2^-32; phi = 2 pi u0,
 * cos(theta) = 1 - u1 (1 - cos(cone)); the new spin is
 * cos(theta) n + sin(theta) (cos(phi) e1 + sin(phi) e2) with
 * e1 = unit(n x r), r = z if |n_z| < 0.9 else x, e2 = n x e1; accepted if
 * u2 < exp(-dE / (k_B T)).  With target_acceptance > 0 the cone follows the
 * feedback of ora_mc_adapt_cone after every sweep. */
typedef struct {
    double T;                  /* K, > 0 */
    double cone_deg;           /* opening angle of the trial cone, degrees (0, 180] (initial, if adaptive) */
    uint64_t seed;
    uint32_t replica;
    double target_acceptance;  /* 0: fixed cone; in (0, 1): adaptive cone toward this acceptance ratio */
} ora_mc_params;

/* Energy change when site i alone changes from n_i to n_new (the terms of
 * the Hamiltonian that contain site i). */
double ora_mc_delta_energy(const ora_system *s, const double *n, int64_t i, const double n_new[3]);
/* The visiting order of sweep `sweep`: a random permutation of 0..N-1. */
void ora_mc_order(int64_t N, uint64_t seed, uint64_t sweep, uint32_t replica, int64_t *order);
/* The cone after a sweep with the given acceptance ratio. */
double ora_mc_adapt_cone(double cone_deg, double acceptance, double target);
/* One sweep with the given cone (sweep counter `sweep`); returns the number
 * of accepted trials, or -1 if the Hamiltonian has a dipole term. */
int64_t ora_mc_sweep(const ora_system *s, double *n, const ora_mc_params *p, double cone_deg, uint64_t sweep);
/* n_sweeps sweeps from sweep0 starting with p->cone_deg; observations every
 * observe_every sweeps; *accepted receives the total accepted trials and
 * *cone_out (may be NULL) the cone after the last sweep.  Returns the
 * number of observations, or -1 as above. */
int64_t ora_mc_run(const ora_system *s, double *n, const ora_mc_params *p, uint64_t sweep0, int64_t n_sweeps,
                   int64_t observe_every, ora_observation *obs, int64_t *accepted, double *cone_out);

/* ------------------------------------------------------------------ GNEB
 * Chain of M images (image-major: image v occupies chain[v*3N .. v*3N+3N),
 * each SoA).  Images 0 and M-1 are fixed. */
enum { ORA_IMAGE_NORMAL = 0, ORA_IMAGE_CLIMBING = 1, ORA_IMAGE_FALLING = 2 };

typedef struct {
    double k_spring;   /* spring constant (meV per rad) */
    double vp_dt;      /* velocity-projection time step */
    double vp_mass;    /* velocity-projection mass */
    const int *image_type;  /* M entries of ORA_IMAGE_*, or NULL (all normal) */
} ora_gneb_params;

/* GNEB forces of every interior image (endpoints get zero force):
 * energies E[M], tangents tau[M*3N] (normalised in 3N, per-spin projected),
 * distances l[M-1] (geodesic, between images v and v+1), forces F[M*3N]. */
void ora_gneb_forces(const ora_system *s, int M, const double *chain, const ora_gneb_params *p,
                     double *E, double *tau, double *l, double *F);
/* n_iter velocity-projection iterations of the whole chain.  v and F_prev
 * (M*3N each) carry the minimiser state between calls; pass F_prev computed
 * by ora_gneb_forces and v = 0 to start. */
void ora_gneb_vp(const ora_system *s, int M, double *chain, double *v, double *F_prev,
                 const ora_gneb_params *p, int n_iter);

/* ------------------------------------- learned dipole field: residual form
 * (not in the paper).  Blocks of B x B cells in the plane and every layer of
 * a one-atom film; block images are [qb][qa][12].  feat: moment M_b[c] at c,
 * first moments Q_b[g][c] = sum_j (r_jg - R_bg) n_jc at 3 + 3 g + c (R_b the
 * block's centroid, Angstrom).  Backbone field (units of C_dd mu^2, i.e.
 * sum_j K(r_j - r_i) n_j with K(r) = (1 - 3 r^ r^)/|r|^3, r in Angstrom):
 * exact over the sites of the blocks within `reach` blocks of i's block
 * along a and b, one dipole M_b at R_b for every other block; u_out holds
 * 3 values per requested site.  Coefficients c0[c] at c, c1[g][c] at
 * 3 + 3 g + c: correction c0 + (r_i - R_b) . c1; ora_ddr_project fits them
 * to a field by least squares per block, ora_ddr_expand evaluates them. */
int ora_ddr_check(const ora_system *s, int B);
void ora_ddr_moments(const ora_system *s, const double *n, int B, double *feat);
void ora_ddr_backbone(const ora_system *s, const double *n, int B, int reach, const int64_t *sites, int64_t n_req,
                      double *u_out);
void ora_ddr_project(const ora_system *s, const double *r, int B, double *coef);
void ora_ddr_expand(const ora_system *s, const double *coef, int B, double *r);

/* ------------------------------------------------- convolutional surrogate
 * Layers of a 3x3 convolution, zero padding, NHWC activations
 * x[B][H][W][Cin], weights w[ky][kx][Cin][Cout], bias b[Cout].  The kernels'
 * contract is reproduced: activations, weights and back-propagated
 * gradients are rounded to bfloat16 (round to nearest even) before they are
 * multiplied; sums are exact (double) here. */
double ora_bf16(double x);
/* on != 0: the conv layers skip the bfloat16 rounding (exact arithmetic). */
void ora_conv_set_exact(int on);
void ora_conv3x3_fwd(int B, int H, int W, int Cin, int Cout, const double *x, const double *w,
                     const double *bias, double *z);
/* dz -> dx (may be NULL), dw, db (accumulated over batch and pixels). */
void ora_conv3x3_bwd(int B, int H, int W, int Cin, int Cout, const double *x, const double *w,
                     const double *dz, double *dx, double *dw, double *db);
/* SiLU y = z / (1 + exp(-z)) and its derivative dy/dz. */
void ora_silu(int64_t n, const double *z, double *y, double *dydz);
/* Adam (Kingma and Ba) step t >= 1 on n parameters. */
void ora_adam(int64_t n, double *p, double *m, double *v, const double *g, double lr, double b1, double b2,
              double eps, int t);

/* OpenMP threads the oracle's parallel loops use, and a way to change them
 * (timing on one core beside all cores). */
int ora_num_threads(void);
void ora_set_num_threads(int n);

/* Physical constants used by the oracle. */
double ora_const_mu_B(void);
double ora_const_k_B(void);
double ora_const_gamma(void);
double ora_const_C_dd(void);

#ifdef __cplusplus
}
#endif
#endif

/*
 * oracle.c -- plain FP64 CPU oracle for the atomistic spin hot path of
 * "Spirit: Multifunctional Framework for Atomistic Spin Simulations"
 * (arXiv:1901.11350).
 *
 * TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
 * baseline of the benchmark call it; the HIP engine never does, and the
 * two share no code.  Built with  gcc -O2 -ffp-contract=off -fopenmp.
 *
 * Sources followed (the paper's text):
 *   - Hamiltonian: Sec. III.A, the extended Heisenberg Hamiltonian equation
 *     (Zeeman, uniaxial anisotropy, exchange and DMI over unique pairs,
 *     dipole-dipole), pairs of any distance: from neighbour shells or as an
 *     explicit list of unique pairs (ora_set_pairs).
 *   - LLG: Sec. III.C, LLG equation terms (i) precession and (ii) damping,
 *     stochastic thermal field with fluctuation-dissipation amplitude and the
 *     1/sqrt(dt) normalisation.
 *   - Depondt's rotation-based Heun scheme: Appendix B (predictor rotates
 *     n(t) by R(A(t)); corrector rotates n(t) by R of the averaged field).
 *   - Energy from fields: Appendix H (linear + quadratic decomposition of H).
 *   - Heun's method and the semi-implicit midpoint scheme SIB: Appendices B
 *     and C (Cramer's rule for each midpoint stage).
 *   - Metropolis Monte Carlo with cone trial moves: Sec. III.B.
 *   - GNEB (improved tangent, geodesic distances, springs, per-spin
 *     projection, velocity projection, climbing and falling images):
 *     Sec. III.D, Appendices D and F; the single-spin Gaussian landscape of
 *     Appendix G as an on-site potential.
 *   - The convolution, SiLU and Adam steps of the learned dipole field (not
 *     in the paper) with the bf16 rounding contract of the GPU kernels.
 * Readings where the paper is silent, garbled or ambiguous are marked
 * "Reading:" next to the code that takes them.  Every function is pinned
 * by a test that does not re-type its formula (tests/test_oracle_*.py).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- constants
 * Reading: the paper prints no unit system.  CODATA 2018 values in
 * meV / Tesla / ps / Angstrom. */
#define J_PER_MEV 1.602176634e-22
#define MU_B_J_PER_T 9.2740100783e-24
#define K_B_J_PER_K 1.380649e-23
#define MU0_OVER_4PI 1.00000000055e-7
#define GAMMA_RAD_PER_PS_T 0.176085963023
#define PI 3.14159265358979323846

#ifdef _OPENMP
#include <omp.h>
int ora_num_threads(void) { return omp_get_max_threads(); }
void ora_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
int ora_num_threads(void) { return 1; }
void ora_set_num_threads(int n) { (void)n; }
#endif

double ora_const_mu_B(void) { return MU_B_J_PER_T / J_PER_MEV; }
double ora_const_k_B(void) { return K_B_J_PER_K / J_PER_MEV; }
double ora_const_gamma(void) { return GAMMA_RAD_PER_PS_T; }
/* mu0/(4 pi) * mu_B^2 / (1 Angstrom)^3, in meV. */
double ora_const_C_dd(void) { return MU0_OVER_4PI * MU_B_J_PER_T * MU_B_J_PER_T / 1e-30 / J_PER_MEV; }

/* ------------------------------------------------------------- small vecs */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------ system */
struct ora_system {
    ora_geometry geo;
    ora_hamiltonian ham;
    int64_t N;
    int n_bonds;
    ora_bond bonds[ORA_MAX_BASIS * ORA_MAX_BONDS_PER_BASIS];
    int n_shell_dist[ORA_MAX_BASIS];
    double shell_dist[ORA_MAX_BASIS][ORA_MAX_SHELLS];
    /* explicit neighbour lists: site i's bonds are nb_j[nb_start[i] .. nb_start[i+1]) */
    int64_t *nb_start;
    int64_t *nb_j;
    int *nb_bond;
    double *pos;   /* 3N cartesian positions in Angstrom (SoA) */
};

static void cell_of(const ora_system *s, int64_t i, int *a, int *b, int *c, int *beta) {
    const int na = s->geo.n_cells[0], nb = s->geo.n_cells[1], nc = s->geo.n_cells[2];
    *a = (int)(i % na);
    *b = (int)((i / na) % nb);
    *c = (int)((i / ((int64_t)na * nb)) % nc);
    *beta = (int)(i / ((int64_t)na * nb * nc));
}

static int64_t site_of(const ora_system *s, int a, int b, int c, int beta) {
    const int64_t na = s->geo.n_cells[0], nb = s->geo.n_cells[1], nc = s->geo.n_cells[2];
    return a + na * (b + nb * (c + nc * (int64_t)beta));
}

/* Cartesian vector (units of the lattice constant) from basis atom bi in a
 * cell to basis atom bj in the cell shifted by (da, db, dc). */
static void bond_vector(const ora_geometry *g, int bi, int bj, int da, int db, int dc, double r[3]) {
    for (int k = 0; k < 3; ++k)
        r[k] = da * g->bravais[0 + k] + db * g->bravais[3 + k] + dc * g->bravais[6 + k]
             + g->basis[3 * bj + k] - g->basis[3 * bi + k];
}

/* Neighbour shells and bonds.  Sec. III.A: exchange/DMI act on unique pairs
 * with no limit on their number or distance; shells are given per shell
 * index.  Reading: for each basis atom, candidate neighbours are sorted by
 * distance; distinct distances (tie tolerance 1e-6 a) are shells 0, 1, 2, ...
 * An axis with a single cell and open boundary carries no translations, so
 * a 2D lattice's shells are in-plane ones. */
static int build_bonds(ora_system *s) {
    const ora_geometry *g = &s->geo;
    const ora_hamiltonian *h = &s->ham;
    const int R = 4;
    int n_shells = h->n_exch > h->n_dmi ? h->n_exch : h->n_dmi;
    int allow[3];
    for (int k = 0; k < 3; ++k) allow[k] = (g->n_cells[k] > 1 || g->periodic[k]) ? R : 0;
    s->n_bonds = 0;
    for (int bi = 0; bi < g->n_basis; ++bi) {
        /* collect distinct distances */
        double dist[ORA_MAX_SHELLS];
        int nd = 0;
        for (int bj = 0; bj < g->n_basis; ++bj)
            for (int da = -allow[0]; da <= allow[0]; ++da)
                for (int db = -allow[1]; db <= allow[1]; ++db)
                    for (int dc = -allow[2]; dc <= allow[2]; ++dc) {
                        double r[3];
                        bond_vector(g, bi, bj, da, db, dc, r);
                        double d = norm3(r);
                        if (d < 1e-6) continue;
                        /* insert d into the sorted list of the ORA_MAX_SHELLS smallest distances */
                        int dup = 0;
                        for (int q = 0; q < nd; ++q)
                            if (fabs(dist[q] - d) < 1e-6) dup = 1;
                        if (dup) continue;
                        if (nd < ORA_MAX_SHELLS) {
                            dist[nd++] = d;
                        } else if (d < dist[nd - 1]) {
                            dist[nd - 1] = d;
                        } else {
                            continue;
                        }
                        for (int q = nd - 1; q > 0 && dist[q] < dist[q - 1]; --q) {
                            double t = dist[q]; dist[q] = dist[q - 1]; dist[q - 1] = t;
                        }
                    }
        s->n_shell_dist[bi] = nd;
        for (int q = 0; q < nd; ++q) s->shell_dist[bi][q] = dist[q];
        if (n_shells > nd) return -1;
        /* emit one directed bond per candidate in the requested shells */
        for (int bj = 0; bj < g->n_basis; ++bj)
            for (int da = -allow[0]; da <= allow[0]; ++da)
                for (int db = -allow[1]; db <= allow[1]; ++db)
                    for (int dc = -allow[2]; dc <= allow[2]; ++dc) {
                        double r[3];
                        bond_vector(g, bi, bj, da, db, dc, r);
                        double d = norm3(r);
                        if (d < 1e-6) continue;
                        int shell = -1;
                        for (int q = 0; q < n_shells; ++q)
                            if (fabs(dist[q] - d) < 1e-6) shell = q;
                        if (shell < 0) continue;
                        if (s->n_bonds >= ORA_MAX_BASIS * ORA_MAX_BONDS_PER_BASIS) return -2;
                        ora_bond *bd = &s->bonds[s->n_bonds++];
                        bd->bi = bi; bd->bj = bj; bd->da = da; bd->db = db; bd->dc = dc;
                        bd->shell = shell;
                        bd->J = shell < h->n_exch ? h->J[shell] : 0.0;
                        double rhat[3] = {r[0] / d, r[1] / d, r[2] / d};
                        double Dm = shell < h->n_dmi ? h->D[shell] : 0.0;
                        /* Reading: the scalar D of a shell becomes a vector along the
                         * bond (bulk) or along z x r_hat (interfacial); D_ji = -D_ij
                         * follows from r_hat_ji = -r_hat_ij. */
                        if (h->dmi_kind == ORA_DMI_BULK) {
                            for (int k = 0; k < 3; ++k) bd->D[k] = Dm * rhat[k];
                        } else {
                            double zhat[3] = {0.0, 0.0, 1.0}, zr[3];
                            cross3(zhat, rhat, zr);
                            for (int k = 0; k < 3; ++k) bd->D[k] = Dm * zr[k];
                        }
                    }
    }
    return 0;
}

/* Site neighbour lists from the bond table.  Reading: periodic axes wrap,
 * open axes drop the bond, and a bond that wraps onto its own site is
 * dropped.  On tiny periodic lattices two translations may reach the same
 * partner; each is a separate pair of the periodic crystal. */
static int build_neighbours(ora_system *s) {
    const int64_t N = s->N;
    s->nb_start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    if (!s->nb_start) return -1;
    int64_t total = 0;
    for (int pass = 0; pass < 2; ++pass) {
        total = 0;
        for (int64_t i = 0; i < N; ++i) {
            int a, b, c, beta;
            cell_of(s, i, &a, &b, &c, &beta);
            if (pass == 0) s->nb_start[i] = total;
            for (int q = 0; q < s->n_bonds; ++q) {
                const ora_bond *bd = &s->bonds[q];
                if (bd->bi != beta) continue;
                int t[3] = {a + bd->da, b + bd->db, c + bd->dc};
                int ok = 1;
                for (int k = 0; k < 3; ++k) {
                    int n_k = s->geo.n_cells[k];
                    if (t[k] < 0 || t[k] >= n_k) {
                        if (s->geo.periodic[k]) {
                            t[k] %= n_k;
                            if (t[k] < 0) t[k] += n_k;
                        } else {
                            ok = 0;
                        }
                    }
                }
                if (!ok) continue;
                int64_t j = site_of(s, t[0], t[1], t[2], bd->bj);
                if (j == i) continue;
                if (pass == 1) {
                    s->nb_j[total] = j;
                    s->nb_bond[total] = q;
                }
                ++total;
            }
        }
        if (pass == 0) {
            s->nb_start[N] = total;
            s->nb_j = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
            s->nb_bond = (int *)malloc(sizeof(int) * (size_t)(total > 0 ? total : 1));
            if (!s->nb_j || !s->nb_bond) return -1;
        }
    }
    return 0;
}

ora_system *ora_create(const ora_geometry *g, const ora_hamiltonian *h) {
    if (g->n_basis < 1 || g->n_basis > ORA_MAX_BASIS) return NULL;
    if (h->n_exch < 0 || h->n_exch > ORA_MAX_SHELLS || h->n_dmi < 0 || h->n_dmi > ORA_MAX_SHELLS) return NULL;
    if (h->n_gauss < 0 || h->n_gauss > ORA_MAX_GAUSS) return NULL;
    for (int k = 0; k < h->n_gauss; ++k)
        if (!(h->gauss_sigma[k] > 0.0) || !(norm3(&h->gauss_c[3 * k]) > 0.0)) return NULL;
    for (int k = 0; k < 3; ++k)
        if (g->n_cells[k] < 1) return NULL;
    ora_system *s = (ora_system *)calloc(1, sizeof(ora_system));
    if (!s) return NULL;
    s->geo = *g;
    s->ham = *h;
    s->N = (int64_t)g->n_cells[0] * g->n_cells[1] * g->n_cells[2] * g->n_basis;
    if (build_bonds(s) != 0 || build_neighbours(s) != 0) {
        ora_destroy(s);
        return NULL;
    }
    s->pos = (double *)malloc(sizeof(double) * 3 * (size_t)s->N);
    if (!s->pos) { ora_destroy(s); return NULL; }
    for (int64_t i = 0; i < s->N; ++i) {
        int a, b, c, beta;
        cell_of(s, i, &a, &b, &c, &beta);
        for (int k = 0; k < 3; ++k) {
            double r = a * g->bravais[k] + b * g->bravais[3 + k] + c * g->bravais[6 + k] + g->basis[3 * beta + k];
            s->pos[k * s->N + i] = r * g->lattice_constant;
        }
    }
    return s;
}

void ora_destroy(ora_system *s) {
    if (!s) return;
    free(s->nb_start);
    free(s->nb_j);
    free(s->nb_bond);
    free(s->pos);
    free(s);
}

int64_t ora_num_sites(const ora_system *s) { return s->N; }

int ora_bonds(const ora_system *s, ora_bond *out, int max_bonds) {
    int n = s->n_bonds < max_bonds ? s->n_bonds : max_bonds;
    memcpy(out, s->bonds, sizeof(ora_bond) * (size_t)n);
    return s->n_bonds;
}

int ora_site_neighbours(const ora_system *s, int64_t i, int64_t *j_out, int *bond_out, int max_out) {
    int64_t deg = s->nb_start[i + 1] - s->nb_start[i];
    for (int64_t q = 0; q < deg && q < max_out; ++q) {
        j_out[q] = s->nb_j[s->nb_start[i] + q];
        bond_out[q] = s->nb_bond[s->nb_start[i] + q];
    }
    return (int)deg;
}

int ora_shell_distances(const ora_system *s, int beta, double *out, int max_out) {
    int n = s->n_shell_dist[beta];
    for (int q = 0; q < n && q < max_out; ++q) out[q] = s->shell_dist[beta][q];
    return n;
}

/* Explicit pairs.  The Hamiltonian's exchange and DMI sums run over unique
 * pairs <ij> of any number and range (Sec. III.A).  Pair p joins basis atom
 * bi[p] of every cell x to basis atom bj[p] of cell x + dcell[p]; as a
 * directed bond table it is kept in both directions, the reverse bond with
 * -D (n_j x n_i = -(n_i x n_j)), so that each site sees its partners and
 * the energy over directed bonds carries the factor 1/2.  The neighbour
 * lists are rebuilt with the same wrap/drop rules as for shells. */
int ora_set_pairs(ora_system *s, int n, const int *bi, const int *bj, const int *dcell, const double *J,
                  const double *D) {
    const int nb = s->geo.n_basis;
    int count[ORA_MAX_BASIS] = {0};
    if (n < 0 || 2 * n > ORA_MAX_BASIS * ORA_MAX_BONDS_PER_BASIS) return -1;
    for (int p = 0; p < n; ++p) {
        const int *d = dcell + 3 * p;
        if (bi[p] < 0 || bi[p] >= nb || bj[p] < 0 || bj[p] >= nb) return -1;
        if (bi[p] == bj[p] && d[0] == 0 && d[1] == 0 && d[2] == 0) return -1;
        for (int q = 0; q < p; ++q) {
            const int *e = dcell + 3 * q;
            int same = bi[q] == bi[p] && bj[q] == bj[p] && e[0] == d[0] && e[1] == d[1] && e[2] == d[2];
            int rev = bi[q] == bj[p] && bj[q] == bi[p] && e[0] == -d[0] && e[1] == -d[1] && e[2] == -d[2];
            if (same || rev) return -1;
        }
        if (++count[bi[p]] > ORA_MAX_BONDS_PER_BASIS || ++count[bj[p]] > ORA_MAX_BONDS_PER_BASIS) return -1;
    }
    s->n_bonds = 0;
    for (int p = 0; p < n; ++p) {
        for (int dir = 0; dir < 2; ++dir) {
            const double sgn = dir == 0 ? 1.0 : -1.0;
            ora_bond *bd = &s->bonds[s->n_bonds++];
            bd->bi = dir == 0 ? bi[p] : bj[p];
            bd->bj = dir == 0 ? bj[p] : bi[p];
            bd->da = (int)sgn * dcell[3 * p];
            bd->db = (int)sgn * dcell[3 * p + 1];
            bd->dc = (int)sgn * dcell[3 * p + 2];
            bd->shell = -1;
            bd->J = J[p];
            for (int k = 0; k < 3; ++k) bd->D[k] = D ? sgn * D[3 * p + k] : 0.0;
        }
    }
    free(s->nb_start);
    free(s->nb_j);
    free(s->nb_bond);
    s->nb_start = NULL;
    s->nb_j = NULL;
    s->nb_bond = NULL;
    return build_neighbours(s) == 0 ? 0 : -2;
}

static int basis_of(const ora_system *s, int64_t i) {
    const int64_t cells = (int64_t)s->geo.n_cells[0] * s->geo.n_cells[1] * s->geo.n_cells[2];
    return (int)(i / cells);
}

static void load(const double *v, int64_t N, int64_t i, double out[3]) {
    out[0] = v[i]; out[1] = v[N + i]; out[2] = v[2 * N + i];
}

/* Dipole-dipole gradient at site i.  Reading: the printed dipole term lacks
 * the factor 3 and has its sign inverted; the textbook dipolar energy
 * 1/2 C_dd sum_{i!=j} mu_i mu_j [n_i.n_j - 3 (n_i.r)(n_j.r)] / r^3 is used,
 * summed over the sites of the sample only (no periodic images).  Its
 * gradient is C_dd mu_i sum_j mu_j [n_j - 3 (n_j.r) r] / r^3. */
static void dipole_gradient_at(const ora_system *s, const double *n, int64_t i, double out[3]) {
    const int64_t N = s->N;
    const double Cdd = ora_const_C_dd();
    double acc[3] = {0.0, 0.0, 0.0};
    double pi[3];
    load(s->pos, N, i, pi);
    for (int64_t j = 0; j < N; ++j) {
        if (j == i) continue;
        double r[3], nj[3];
        load(s->pos, N, j, r);
        for (int k = 0; k < 3; ++k) r[k] -= pi[k];
        double d = norm3(r);
        double rh[3] = {r[0] / d, r[1] / d, r[2] / d};
        load(n, N, j, nj);
        double mu_j = s->ham.mu[basis_of(s, j)];
        double nr = dot3(nj, rh);
        double inv_r3 = 1.0 / (d * d * d);
        for (int k = 0; k < 3; ++k) acc[k] += mu_j * (nj[k] - 3.0 * nr * rh[k]) * inv_r3;
    }
    double mu_i = s->ham.mu[basis_of(s, i)];
    for (int k = 0; k < 3; ++k) out[k] = Cdd * mu_i * acc[k];
}

void ora_dipole_gradient_sites(const ora_system *s, const double *n, const int64_t *sites,
                               int64_t n_req, double *g_out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_req; ++q) dipole_gradient_at(s, n, sites[q], g_out + 3 * q);
}

/* Gaussian on-site potentials (Appendix G): energy of one spin and its
 * gradient  d/dn a exp(-(1 - n.c)^2 / (2 s^2)) = a exp(...) (1 - n.c) / s^2 c.
 * Reading: the centres c_k are directions (normalised here); the printed
 * table lists them unnormalised. */
static void gauss_centre(const ora_system *s, int k, double c[3]) {
    const double *ck = &s->ham.gauss_c[3 * k];
    const double r = norm3(ck);
    for (int q = 0; q < 3; ++q) c[q] = ck[q] / r;
}

static double gauss_energy(const ora_system *s, const double n[3]) {
    double e = 0.0;
    for (int k = 0; k < s->ham.n_gauss; ++k) {
        double c[3];
        gauss_centre(s, k, c);
        const double d = 1.0 - dot3(n, c), sg = s->ham.gauss_sigma[k];
        e += s->ham.gauss_a[k] * exp(-d * d / (2.0 * sg * sg));
    }
    return e;
}

static void gauss_gradient_add(const ora_system *s, const double n[3], double g[3]) {
    for (int k = 0; k < s->ham.n_gauss; ++k) {
        double c[3];
        gauss_centre(s, k, c);
        const double d = 1.0 - dot3(n, c), sg = s->ham.gauss_sigma[k];
        const double f = s->ham.gauss_a[k] * exp(-d * d / (2.0 * sg * sg)) * d / (sg * sg);
        for (int q = 0; q < 3; ++q) g[q] += f * c[q];
    }
}

/* Gradient dH/dn_i of the Hamiltonian (Sec. III.A) in the embedding space:
 *   Zeeman      -mu_i mu_B B
 *   anisotropy  -2 K (K_hat . n_i) K_hat
 *   exchange    -sum_j J_ij n_j
 *   DMI         -sum_j n_j x D_ij        (from d/dn_i [D.(n_i x n_j)] = n_j x D)
 *   dipole      see dipole_gradient_at. */
void ora_gradient(const ora_system *s, const double *n, double *g, double *terms) {
    const int64_t N = s->N;
    const double muB = ora_const_mu_B();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int beta = basis_of(s, i);
        double ni[3];
        load(n, N, i, ni);
        double gz[3], gk[3], gj[3] = {0, 0, 0}, gd[3] = {0, 0, 0}, gdd[3] = {0, 0, 0};
        for (int k = 0; k < 3; ++k) gz[k] = -s->ham.mu[beta] * muB * s->ham.B[k];
        const double *ax = &s->ham.K_axis[3 * beta];
        double kn = dot3(ax, ni);
        for (int k = 0; k < 3; ++k) gk[k] = -2.0 * s->ham.K[beta] * kn * ax[k];
        gauss_gradient_add(s, ni, gk);
        for (int64_t q = s->nb_start[i]; q < s->nb_start[i + 1]; ++q) {
            const ora_bond *bd = &s->bonds[s->nb_bond[q]];
            double nj[3], c[3];
            load(n, N, s->nb_j[q], nj);
            cross3(nj, bd->D, c);
            for (int k = 0; k < 3; ++k) {
                gj[k] -= bd->J * nj[k];
                gd[k] -= c[k];
            }
        }
        if (s->ham.ddi) dipole_gradient_at(s, n, i, gdd);
        for (int k = 0; k < 3; ++k) g[k * N + i] = gz[k] + gk[k] + gj[k] + gd[k] + gdd[k];
        if (terms) {
            for (int k = 0; k < 3; ++k) {
                terms[0 * 3 * N + k * N + i] = gz[k];
                terms[1 * 3 * N + k * N + i] = gk[k];
                terms[2 * 3 * N + k * N + i] = gj[k];
                terms[3 * 3 * N + k * N + i] = gd[k];
                terms[4 * 3 * N + k * N + i] = gdd[k];
            }
        }
    }
}

/* Energy by the definition of the Hamiltonian (Sec. III.A).  The unique-pair
 * sums of exchange and DMI are taken as 1/2 of the sums over directed bonds
 * (every unique pair appears once from each side). */
double ora_energy(const ora_system *s, const double *n, double *per_term) {
    const int64_t N = s->N;
    const double muB = ora_const_mu_B();
    const double Cdd = ora_const_C_dd();
    double ez = 0.0, ek = 0.0, ej = 0.0, ed = 0.0, edd = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : ez, ek, ej, ed, edd)
    for (int64_t i = 0; i < N; ++i) {
        int beta = basis_of(s, i);
        double ni[3];
        load(n, N, i, ni);
        ez += -s->ham.mu[beta] * muB * dot3(s->ham.B, ni);
        double kn = dot3(&s->ham.K_axis[3 * beta], ni);
        ek += -s->ham.K[beta] * kn * kn + gauss_energy(s, ni);
        for (int64_t q = s->nb_start[i]; q < s->nb_start[i + 1]; ++q) {
            const ora_bond *bd = &s->bonds[s->nb_bond[q]];
            double nj[3], c[3];
            load(n, N, s->nb_j[q], nj);
            cross3(ni, nj, c);
            ej += -0.5 * bd->J * dot3(ni, nj);
            ed += -0.5 * dot3(bd->D, c);
        }
        if (s->ham.ddi) {
            double pi[3];
            load(s->pos, N, i, pi);
            for (int64_t j = 0; j < N; ++j) {
                if (j == i) continue;
                double r[3], nj[3];
                load(s->pos, N, j, r);
                for (int k = 0; k < 3; ++k) r[k] -= pi[k];
                double d = norm3(r);
                double rh[3] = {r[0] / d, r[1] / d, r[2] / d};
                load(n, N, j, nj);
                double mm = s->ham.mu[beta] * s->ham.mu[basis_of(s, j)];
                edd += 0.5 * Cdd * mm * (dot3(ni, nj) - 3.0 * dot3(ni, rh) * dot3(nj, rh)) / (d * d * d);
            }
        }
    }
    if (per_term) {
        per_term[0] = ez; per_term[1] = ek; per_term[2] = ej; per_term[3] = ed; per_term[4] = edd;
    }
    return ez + ek + ej + ed + edd;
}

/* ------------------------------------------------------------------ Philox
 * Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw (SC'11):
 * each round multiplies counter words 0 and 2 by the round multipliers
 * (full 64-bit products), permutes and xors with the key; the key is
 * incremented by the Weyl constants between rounds. */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Sec. III.C: eta_i holds three independent standard normals per step.
 * Reading: uniforms u_k = (x_k + 1/2) 2^-32 from one Philox block, then the
 * Box-Muller transform on (u0, u1) and (u2, u3); the first three normals
 * are used. */
void ora_thermal_normals(uint64_t seed, uint64_t step, uint32_t site, uint32_t replica, double eta[3]) {
    uint32_t ctr[4] = {site, (uint32_t)step, (uint32_t)(step >> 32), replica};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    ora_philox4x32_10(ctr, key, x);
    double u[4];
    for (int k = 0; k < 4; ++k) u[k] = ((double)x[k] + 0.5) * (1.0 / 4294967296.0);
    double r0 = sqrt(-2.0 * log(u[0]));
    double r1 = sqrt(-2.0 * log(u[2]));
    eta[0] = r0 * cos(2.0 * PI * u[1]);
    eta[1] = r0 * sin(2.0 * PI * u[1]);
    eta[2] = r1 * cos(2.0 * PI * u[3]);
}

/* ------------------------------------------------------------------ LLG */

/* Rotation of n about omega by the angle |omega| dt (Rodrigues' formula).
 * Reading: the rotation matrix R(A) of Appendix B is not printed; with
 * dn/dt = n x A = (-A) x n the exact motion for constant A is a rotation
 * about omega = -A at angular speed |A|. */
void ora_rotate(const double n[3], const double omega[3], double dt, double out[3]) {
    double w = norm3(omega);
    double theta = w * dt;
    if (theta < 1e-12) {
        /* second-order Taylor form of the same rotation */
        double c1[3], c2[3];
        cross3(omega, n, c1);
        cross3(omega, c1, c2);
        for (int k = 0; k < 3; ++k) out[k] = n[k] + c1[k] * dt + 0.5 * c2[k] * dt * dt;
        return;
    }
    double e[3] = {omega[0] / w, omega[1] / w, omega[2] / w};
    double exn[3];
    cross3(e, n, exn);
    double en = dot3(e, n);
    double ct = cos(theta), st = sin(theta);
    for (int k = 0; k < 3; ++k) out[k] = n[k] * ct + exn[k] * st + e[k] * en * (1.0 - ct);
}

/* A_i of the LLG equation written as dn/dt = n x A (Appendix B), terms (i)
 * precession and (ii) damping of Sec. III.C:
 *   A = -gamma/(1+alpha^2) (B + alpha n x B),  B in Tesla.
 * Reading: B_eff = -dH/dn is an energy; dividing by mu_i mu_B gives Tesla,
 * which is what the 1/mu_i of the printed prefactor expresses. */
static void llg_A(const double n[3], const double Bt[3], double alpha, double A[3]) {
    const double gp = ora_const_gamma() / (1.0 + alpha * alpha);
    double nxB[3];
    cross3(n, Bt, nxB);
    for (int k = 0; k < 3; ++k) A[k] = -gp * (Bt[k] + alpha * nxB[k]);
}

/* Thermal field amplitude in Tesla per component (Sec. III.C):
 * sqrt(2 alpha k_B T / (gamma mu_i mu_B)) / sqrt(dt). */
static double thermal_sigma(double alpha, double T, double mu, double dt) {
    if (T <= 0.0) return 0.0;
    return sqrt(2.0 * alpha * ora_const_k_B() * T / (ora_const_gamma() * mu * ora_const_mu_B() * dt));
}

/* Depondt's scheme (Appendix B):
 *   n^p = R(A(n)) n;   A^c = (A(n) + A(n^p)) / 2;   n(t+dt) = R(A^c) n.
 * Reading: the same thermal normals enter predictor and corrector
 * (stochastic Heun); rotation keeps |n| so no renormalisation is applied. */
void ora_depondt_step(const ora_system *s, double *n, const ora_llg_params *p, uint64_t step) {
    const int64_t N = s->N;
    const double muB = ora_const_mu_B();
    double *g = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *np_ = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *A = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *Bth = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    ora_gradient(s, n, g, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double mu = s->ham.mu[basis_of(s, i)];
        double sigma = thermal_sigma(p->alpha, p->T, mu, p->dt);
        double eta[3] = {0.0, 0.0, 0.0};
        if (sigma > 0.0) ora_thermal_normals(p->seed, step, (uint32_t)i, p->replica, eta);
        double ni[3], Bt[3], Ai[3], w[3], out[3];
        load(n, N, i, ni);
        for (int k = 0; k < 3; ++k) {
            Bth[k * N + i] = sigma * eta[k];
            Bt[k] = -g[k * N + i] / (mu * muB) + Bth[k * N + i];
        }
        llg_A(ni, Bt, p->alpha, Ai);
        for (int k = 0; k < 3; ++k) {
            A[k * N + i] = Ai[k];
            w[k] = -Ai[k];
        }
        ora_rotate(ni, w, p->dt, out);
        for (int k = 0; k < 3; ++k) np_[k * N + i] = out[k];
    }
    ora_gradient(s, np_, g, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double mu = s->ham.mu[basis_of(s, i)];
        double npi[3], ni[3], Bt[3], Ap[3], w[3], out[3];
        load(np_, N, i, npi);
        load(n, N, i, ni);
        for (int k = 0; k < 3; ++k) Bt[k] = -g[k * N + i] / (mu * muB) + Bth[k * N + i];
        llg_A(npi, Bt, p->alpha, Ap);
        for (int k = 0; k < 3; ++k) w[k] = -0.5 * (A[k * N + i] + Ap[k]);
        ora_rotate(ni, w, p->dt, out);
        for (int k = 0; k < 3; ++k) n[k * N + i] = out[k];
    }
    free(g);
    free(np_);
    free(A);
    free(Bth);
}

/* Effective field in Tesla of every site with its thermal part:
 * Bt_i = -g_i / (mu_i mu_B) + sigma_i eta_i (eta drawn at `step`). */
static void field_tesla(const ora_system *s, const double *n, const ora_llg_params *p, uint64_t step,
                        double *g, double *Bt) {
    const int64_t N = s->N;
    const double muB = ora_const_mu_B();
    ora_gradient(s, n, g, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double mu = s->ham.mu[basis_of(s, i)];
        double sigma = thermal_sigma(p->alpha, p->T, mu, p->dt);
        double eta[3] = {0.0, 0.0, 0.0};
        if (sigma > 0.0) ora_thermal_normals(p->seed, step, (uint32_t)i, p->replica, eta);
        for (int k = 0; k < 3; ++k) Bt[k * N + i] = -g[k * N + i] / (mu * muB) + sigma * eta[k];
    }
}

/* Heun's method (Appendix B, first part) for dn/dt = f(n) = n x A(n):
 *   n^p = n + dt f(n);   n(t+dt) = n + dt (f(n) + f(n^p)) / 2.
 * Readings: the same thermal normals in both stages; the scheme does not
 * keep |n|, and both n^p and n(t+dt) are renormalised at every step (with
 * this choice the single-spin precession of Sec. III.C, B = 1 T, alpha = 0.1,
 * dt = 10 fs, stays within the 1e-6 of the exact solution the paper quotes
 * for Heun's method; without renormalising n^p it does not). */
void ora_heun_step(const ora_system *s, double *n, const ora_llg_params *p, uint64_t step) {
    const int64_t N = s->N;
    double *g = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *Bt = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *np_ = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *f0 = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    field_tesla(s, n, p, step, g, Bt);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double ni[3], Bi[3], Ai[3], fi[3];
        load(n, N, i, ni);
        load(Bt, N, i, Bi);
        llg_A(ni, Bi, p->alpha, Ai);
        cross3(ni, Ai, fi);
        double pi[3];
        for (int k = 0; k < 3; ++k) {
            f0[k * N + i] = fi[k];
            pi[k] = ni[k] + p->dt * fi[k];
        }
        const double r = norm3(pi);
        for (int k = 0; k < 3; ++k) np_[k * N + i] = pi[k] / r;
    }
    field_tesla(s, np_, p, step, g, Bt);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double ni[3], npi[3], Bi[3], Ap[3], fp[3], out[3];
        load(n, N, i, ni);
        load(np_, N, i, npi);
        load(Bt, N, i, Bi);
        llg_A(npi, Bi, p->alpha, Ap);
        cross3(npi, Ap, fp);
        for (int k = 0; k < 3; ++k) out[k] = ni[k] + 0.5 * p->dt * (f0[k * N + i] + fp[k]);
        const double r = norm3(out);
        for (int k = 0; k < 3; ++k) n[k * N + i] = out[k] / r;
    }
    free(g);
    free(Bt);
    free(np_);
    free(f0);
}

/* Solution x of (I + skew(w)) x = a by Cramer's rule (Appendix C):
 * M = [[1, -wz, wy], [wz, 1, -wx], [-wy, wx, 1]], x_k = det(M^k) / det(M),
 * M^k = M with column k replaced by a. */
static double det3(const double m[9]) {
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
           m[2] * (m[3] * m[7] - m[4] * m[6]);
}

static void sib_solve(const double w[3], const double a[3], double x[3]) {
    const double M[9] = {1.0, -w[2], w[1], w[2], 1.0, -w[0], -w[1], w[0], 1.0};
    const double d = det3(M);
    for (int k = 0; k < 3; ++k) {
        double Mk[9];
        for (int q = 0; q < 9; ++q) Mk[q] = M[q];
        for (int r = 0; r < 3; ++r) Mk[3 * r + k] = a[r];
        x[k] = det3(Mk) / d;
    }
}

/* One implicit-midpoint stage with a frozen field: the x solving
 * x = n + dt (n + x)/2 x A, i.e. (I + skew(w)) x = n + n x w, w = dt A / 2.
 * Reading: the printed matrix M carries A; consistency with the midpoint
 * equation it solves requires A dt / 2. */
static void sib_stage(const double n[3], const double A[3], double dt, double x[3]) {
    double w[3], nxw[3], a[3];
    for (int k = 0; k < 3; ++k) w[k] = 0.5 * dt * A[k];
    cross3(n, w, nxw);
    for (int k = 0; k < 3; ++k) a[k] = n[k] + nxw[k];
    sib_solve(w, a, x);
}

/* Semi-implicit scheme B (Appendix C): predictor with A(t, {n}), corrector
 * with A at the midpoint spins m = (n + n^p)/2 (also in the damping term of
 * site i).  Readings: the same thermal normals in both stages; m is not
 * renormalised; the midpoint structure keeps |n|, no renormalisation. */
void ora_sib_step(const ora_system *s, double *n, const ora_llg_params *p, uint64_t step) {
    const int64_t N = s->N;
    double *g = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *Bt = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *m = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    field_tesla(s, n, p, step, g, Bt);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double ni[3], Bi[3], Ai[3], npi[3];
        load(n, N, i, ni);
        load(Bt, N, i, Bi);
        llg_A(ni, Bi, p->alpha, Ai);
        sib_stage(ni, Ai, p->dt, npi);
        for (int k = 0; k < 3; ++k) m[k * N + i] = 0.5 * (ni[k] + npi[k]);
    }
    field_tesla(s, m, p, step, g, Bt);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double ni[3], mi[3], Bi[3], Am[3], out[3];
        load(n, N, i, ni);
        load(m, N, i, mi);
        load(Bt, N, i, Bi);
        llg_A(mi, Bi, p->alpha, Am);
        sib_stage(ni, Am, p->dt, out);
        for (int k = 0; k < 3; ++k) n[k * N + i] = out[k];
    }
    free(g);
    free(Bt);
    free(m);
}

void ora_llg_step(const ora_system *s, double *n, const ora_llg_params *p, uint64_t step) {
    if (p->solver == ORA_SOLVER_HEUN)
        ora_heun_step(s, n, p, step);
    else if (p->solver == ORA_SOLVER_SIB)
        ora_sib_step(s, n, p, step);
    else
        ora_depondt_step(s, n, p, step);
}

/* Observables: energy with per-term split, maximum torque |n x dH/dn|,
 * mean spin, maximum deviation of |n| from 1. */
void ora_observe(const ora_system *s, const double *n, int64_t step, ora_observation *obs) {
    const int64_t N = s->N;
    double *g = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    ora_gradient(s, n, g, NULL);
    obs->step = step;
    obs->E = ora_energy(s, n, obs->per_term);
    double tmax = 0.0, M[3] = {0, 0, 0}, dev = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double ni[3], gi[3], t[3];
        load(n, N, i, ni);
        load(g, N, i, gi);
        cross3(ni, gi, t);
        double tn = norm3(t);
        if (!(tn <= tmax)) tmax = tn; /* propagates NaN */
        for (int k = 0; k < 3; ++k) M[k] += ni[k];
        double dn = fabs(norm3(ni) - 1.0);
        if (dn > dev) dev = dn;
    }
    obs->max_torque = tmax;
    for (int k = 0; k < 3; ++k) obs->M[k] = M[k] / (double)N;
    obs->max_norm_dev = dev;
    free(g);
}

int64_t ora_run(const ora_system *s, double *n, const ora_llg_params *p, uint64_t step0,
                int64_t n_steps, int64_t observe_every, ora_observation *obs) {
    int64_t n_obs = 0;
    for (int64_t t = 0; t < n_steps; ++t) {
        ora_llg_step(s, n, p, step0 + (uint64_t)t);
        if (observe_every > 0 && (t + 1) % observe_every == 0 && obs)
            ora_observe(s, n, (int64_t)step0 + t + 1, &obs[n_obs++]);
    }
    return n_obs;
}

/* ----------------------------------------------------------- Monte Carlo */

double ora_mc_delta_energy(const ora_system *s, const double *n, int64_t i, const double n_new[3]) {
    const int64_t N = s->N;
    const int beta = basis_of(s, i);
    const double muB = ora_const_mu_B();
    double ni[3], dn[3];
    load(n, N, i, ni);
    for (int k = 0; k < 3; ++k) dn[k] = n_new[k] - ni[k];
    /* Zeeman and the pair terms are linear in n_i: their change is
     * dn . (coefficient of n_i) */
    double lin[3];
    for (int k = 0; k < 3; ++k) lin[k] = -s->ham.mu[beta] * muB * s->ham.B[k];
    for (int64_t q = s->nb_start[i]; q < s->nb_start[i + 1]; ++q) {
        const ora_bond *bd = &s->bonds[s->nb_bond[q]];
        double nj[3], c[3];
        load(n, N, s->nb_j[q], nj);
        cross3(nj, bd->D, c);
        for (int k = 0; k < 3; ++k) lin[k] -= bd->J * nj[k] + c[k];
    }
    const double *ax = &s->ham.K_axis[3 * beta];
    const double k_old = dot3(ax, ni), k_new = dot3(ax, n_new);
    return dot3(dn, lin) - s->ham.K[beta] * (k_new * k_new - k_old * k_old) + gauss_energy(s, n_new) -
           gauss_energy(s, ni);
}

/* The Metropolis sweep of Sec. III.B: every spin is picked once, one after
 * the other, in an order drawn at random for each sweep, and given a trial
 * step inside a cone about its current direction.  Needs no dipole term
 * (its energy change is not local); any lattice and basis. */
static int mc_admissible(const ora_system *s) { return !s->ham.ddi; }

/* Trial direction (Sec. III.B): the current spin is the z axis of a local
 * frame; phi uniform in [0, 2 pi), cos(theta) uniform in [cos(cone), 1].
 * Reading: the frame is e1 = unit(n x r), r = z if |n_z| < 0.9 else x,
 * e2 = n x e1 (any frame gives the same distribution of trials). */
static void mc_trial(const double n[3], const double u[4], double cos_cone, double out[3]) {
    double r[3] = {0.0, 0.0, 0.0}, e1[3], e2[3];
    if (fabs(n[2]) < 0.9) r[2] = 1.0; else r[0] = 1.0;
    cross3(n, r, e1);
    const double l = norm3(e1);
    for (int k = 0; k < 3; ++k) e1[k] /= l;
    cross3(n, e1, e2);
    const double phi = 2.0 * PI * u[0];
    const double ct = 1.0 - u[1] * (1.0 - cos_cone);
    const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    for (int k = 0; k < 3; ++k) out[k] = ct * n[k] + st * (cos(phi) * e1[k] + sin(phi) * e2[k]);
}

/* Visiting order of one sweep: a uniformly random permutation of the N
 * sites (Fisher-Yates).  Reading: its random integers come from Philox
 * blocks of counter (2^31 + k, s_lo, s_hi, replica), key (seed_lo, seed_hi)
 * -- counters the trial draws (word 0 = site < 2^31) never use; step k
 * swaps position k with position floor(r (k + 1) / 2^64), r = the block's
 * first two words as one 64-bit integer. */
void ora_mc_order(int64_t N, uint64_t seed, uint64_t sweep, uint32_t replica, int64_t *order) {
    for (int64_t i = 0; i < N; ++i) order[i] = i;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t k = N - 1; k > 0; --k) {
        const uint32_t ctr[4] = {0x80000000u + (uint32_t)k, (uint32_t)sweep, (uint32_t)(sweep >> 32), replica};
        uint32_t x[4];
        ora_philox4x32_10(ctr, key, x);
        const uint64_t r = ((uint64_t)x[0] << 32) | x[1];
        const int64_t j = (int64_t)(((unsigned __int128)r * (uint64_t)(k + 1)) >> 64);
        const int64_t t = order[k];
        order[k] = order[j];
        order[j] = t;
    }
}

int64_t ora_mc_sweep(const ora_system *s, double *n, const ora_mc_params *p, double cone_deg, uint64_t sweep) {
    if (!mc_admissible(s)) return -1;
    const int64_t N = s->N;
    const double kT = ora_const_k_B() * p->T;
    const double cos_cone = cos(cone_deg * PI / 180.0);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    ora_mc_order(N, p->seed, sweep, p->replica, order);
    int64_t accepted = 0;
    for (int64_t v = 0; v < N; ++v) {   /* sequential: each trial sees every earlier move */
        const int64_t i = order[v];
        const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)sweep, (uint32_t)(sweep >> 32), p->replica};
        const uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
        uint32_t x[4];
        ora_philox4x32_10(ctr, key, x);
        double u[4];
        for (int k = 0; k < 4; ++k) u[k] = ((double)x[k] + 0.5) * (1.0 / 4294967296.0);
        double ni[3], nn[3];
        load(n, N, i, ni);
        mc_trial(ni, u, cos_cone, nn);
        const double dE = ora_mc_delta_energy(s, n, i, nn);
        /* accepted with probability min(1, exp(-dE / k_B T)) */
        if (u[2] < exp(-dE / kT)) {
            for (int k = 0; k < 3; ++k) n[k * N + i] = nn[k];
            ++accepted;
        }
    }
    free(order);
    return accepted;
}

/* Adaptive cone (Sec. III.B: the cone angle follows a feedback loop toward
 * a desired acceptance ratio; the loop is not printed).  Reading: after
 * every sweep with acceptance ratio a, cone <- min(180, cone (1 + a - a*))
 * degrees: wider while more than the target a* is accepted, narrower
 * while fewer; the factor lies in [1 - a*, 2 - a*], so the cone never
 * reaches zero. */
double ora_mc_adapt_cone(double cone_deg, double acceptance, double target) {
    if (!(target > 0.0)) return cone_deg;
    const double c = cone_deg * (1.0 + acceptance - target);
    return c > 180.0 ? 180.0 : c;
}

int64_t ora_mc_run(const ora_system *s, double *n, const ora_mc_params *p, uint64_t sweep0, int64_t n_sweeps,
                   int64_t observe_every, ora_observation *obs, int64_t *accepted, double *cone_out) {
    int64_t n_obs = 0, acc = 0;
    double cone = p->cone_deg;
    for (int64_t t = 0; t < n_sweeps; ++t) {
        const int64_t a = ora_mc_sweep(s, n, p, cone, sweep0 + (uint64_t)t);
        if (a < 0) return -1;
        acc += a;
        cone = ora_mc_adapt_cone(cone, s->N > 0 ? (double)a / (double)s->N : 0.0, p->target_acceptance);
        if (observe_every > 0 && (t + 1) % observe_every == 0 && obs)
            ora_observe(s, n, (int64_t)sweep0 + t + 1, &obs[n_obs++]);
    }
    if (accepted) *accepted = acc;
    if (cone_out) *cone_out = cone;
    return n_obs;
}

/* ------------------------------------------------------------------ GNEB
 * Geodesic nudged elastic band (Sec. III.D, Appendices D and F). */

/* Great-circle angle between two unit vectors. */
static double geodesic_angle(const double a[3], const double b[3]) {
    double c[3];
    cross3(a, b, c);
    return atan2(norm3(c), dot3(a, b));
}

void ora_gneb_forces(const ora_system *s, int M, const double *chain, const ora_gneb_params *p,
                     double *E, double *tau, double *l, double *F) {
    const int64_t N = s->N, L = 3 * N;
    double *g = (double *)malloc(sizeof(double) * (size_t)L);
    for (int v = 0; v < M; ++v) E[v] = ora_energy(s, chain + v * L, NULL);
    /* geodesic distance between neighbouring images (Appendix F): the
     * Euclidean norm of the per-spin great-circle angles */
    for (int v = 0; v + 1 < M; ++v) {
        double acc = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double a[3], b[3];
            load(chain + v * L, N, i, a);
            load(chain + (v + 1) * L, N, i, b);
            double t = geodesic_angle(a, b);
            acc += t * t;
        }
        l[v] = sqrt(acc);
    }
    for (int v = 0; v < M; ++v) {
        double *tv = tau + v * L, *Fv = F + v * L;
        if (v == 0 || v == M - 1) {
            for (int64_t k = 0; k < L; ++k) { tv[k] = 0.0; Fv[k] = 0.0; }
            continue;
        }
        const double *xm = chain + (v - 1) * L, *x0 = chain + v * L, *xp = chain + (v + 1) * L;
        /* Reading: the tangent rule the paper cites (Henkelman and Jonsson's
         * improved tangent) is not printed; its published form is used: the
         * difference towards the higher-energy neighbour, and at an energy
         * extremum an energy-weighted mix of both differences. */
        const double Ep = E[v + 1], E0 = E[v], Em = E[v - 1];
        double wp, wm;
        if (Ep > E0 && E0 > Em) {
            wp = 1.0; wm = 0.0;
        } else if (Ep < E0 && E0 < Em) {
            wp = 0.0; wm = 1.0;
        } else {
            double d1 = fabs(Ep - E0), d2 = fabs(Em - E0);
            double dmax = d1 > d2 ? d1 : d2, dmin = d1 > d2 ? d2 : d1;
            if (Ep > Em) { wp = dmax; wm = dmin; } else { wp = dmin; wm = dmax; }
        }
        for (int64_t k = 0; k < L; ++k) tv[k] = wp * (xp[k] - x0[k]) + wm * (x0[k] - xm[k]);
        /* project onto the tangent plane of each spin, then normalise in 3N
         * (Appendix F) */
        double nrm = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double n[3], t[3];
            load(x0, N, i, n);
            load(tv, N, i, t);
            double tn = dot3(t, n);
            for (int c = 0; c < 3; ++c) tv[c * N + i] = t[c] - tn * n[c];
        }
        for (int64_t k = 0; k < L; ++k) nrm += tv[k] * tv[k];
        nrm = sqrt(nrm);
        if (nrm > 0.0)
            for (int64_t k = 0; k < L; ++k) tv[k] /= nrm;
        /* energy force -grad E + (grad E . tau) tau, per-spin projected, plus
         * the spring force.  Reading: the printed spring force
         * (l_{v-1,v} - l_{v,v+1}) tau carries no spring constant and the sign
         * that would push images apart; the usual form
         * k (l_{v,v+1} - l_{v-1,v}) tau, which equalises the distances, is used. */
        ora_gradient(s, x0, g, NULL);
        double gt = 0.0;
        for (int64_t k = 0; k < L; ++k) gt += g[k] * tv[k];
        /* climbing image (Sec. III.D): no spring, the gradient component
         * along the path inverted, F = -grad E + 2 (grad E . tau) tau.
         * Falling image: no spring, F = -grad E, so it relaxes into the
         * nearest minimum.  Reading: the paper names the falling image but
         * prints no force for it; the full energy force is its natural
         * counterpart. */
        const int type = p->image_type ? p->image_type[v] : ORA_IMAGE_NORMAL;
        const double cpar = type == ORA_IMAGE_CLIMBING ? 2.0 : (type == ORA_IMAGE_FALLING ? 0.0 : 1.0);
        const double fs = type == ORA_IMAGE_NORMAL ? p->k_spring * (l[v] - l[v - 1]) : 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double n[3], fe[3];
            load(x0, N, i, n);
            for (int c = 0; c < 3; ++c) fe[c] = -g[c * N + i] + cpar * gt * tv[c * N + i];
            double fn = dot3(fe, n);
            for (int c = 0; c < 3; ++c) Fv[c * N + i] = fe[c] - fn * n[c] + fs * tv[c * N + i];
        }
    }
    free(g);
}

/* Velocity projection (Appendix D): Verlet steps of massive particles with
 * force F, the velocity projected on the force (3N-dimensional over the
 * whole chain; zeroed when it points against the force), spins renormalised
 * after every position update. */
void ora_gneb_vp(const ora_system *s, int M, double *chain, double *v, double *F_prev,
                 const ora_gneb_params *p, int n_iter) {
    const int64_t N = s->N, L = 3 * N;
    const double dt = p->vp_dt, m = p->vp_mass;
    double *E = (double *)malloc(sizeof(double) * (size_t)M);
    double *l = (double *)malloc(sizeof(double) * (size_t)(M > 1 ? M - 1 : 1));
    double *tau = (double *)malloc(sizeof(double) * (size_t)(M * L));
    double *F = (double *)malloc(sizeof(double) * (size_t)(M * L));
    for (int it = 0; it < n_iter; ++it) {
        for (int im = 1; im + 1 < M; ++im) {
            double *x = chain + im * L, *vv = v + im * L, *fp = F_prev + im * L;
            for (int64_t k = 0; k < L; ++k) x[k] = x[k] + dt * vv[k] + dt * dt / (2.0 * m) * fp[k];
            for (int64_t i = 0; i < N; ++i) {
                double n[3];
                load(x, N, i, n);
                double r = norm3(n);
                for (int c = 0; c < 3; ++c) x[c * N + i] = n[c] / r;
            }
        }
        ora_gneb_forces(s, M, chain, p, E, tau, l, F);
        double vf = 0.0, ff = 0.0;
        for (int64_t k = 0; k < M * L; ++k) {
            v[k] = v[k] + dt / (2.0 * m) * (F_prev[k] + F[k]);
            vf += v[k] * F[k];
            ff += F[k] * F[k];
        }
        const double scale = (vf > 0.0 && ff > 0.0) ? vf / ff : 0.0;
        for (int64_t k = 0; k < M * L; ++k) {
            v[k] = scale * F[k];
            F_prev[k] = F[k];
        }
    }
    free(E);
    free(l);
    free(tau);
    free(F);
}

/* ------------------------------------- learned dipole field: residual form
 * (not in the paper; a stand-in for its costliest term, the dipolar sum of
 * Sec. III.A).  Sites of a one-atom film are grouped into blocks of B x B
 * cells in the plane and every layer.  Block b (pixel (qa, qb) of the block
 * grid) has the centroid R_b of its sites, the moment M_b = sum_j n_j and
 * the first moments Q_b[g][c] = sum_j (r_jg - R_bg) n_jc.  The backbone
 * field of site i, in units of C_dd mu^2 (u = sum_j K(r_j - r_i) n_j,
 * K(r) = (1 - 3 r^ r^) / |r|^3, r in Angstrom), is summed exactly over the
 * sites of the blocks within `reach` blocks of i's block along a and b, and
 * takes every other block as the single dipole M_b at R_b.  The learned
 * part corrects it per block by c0_b + (r_i - R_b) . c1_b (12 coefficients:
 * c0[c], then c1[g][c] at 3 + 3 g + c); block images are [qb][qa][12]. */

static void block_of(const ora_system *s, int64_t i, int B, int *qa, int *qb) {
    int a, b, c, beta;
    cell_of(s, i, &a, &b, &c, &beta);
    *qa = a / B;
    *qb = b / B;
}

int ora_ddr_check(const ora_system *s, int B) {
    if (s->geo.n_basis != 1 || B < 1) return -1;
    if (s->geo.n_cells[0] % B || s->geo.n_cells[1] % B) return -1;
    return 0;
}

/* centroids R_b (Angstrom), [qb][qa][3] */
static void block_centroids(const ora_system *s, int B, double *R) {
    const int nba = s->geo.n_cells[0] / B, nbb = s->geo.n_cells[1] / B;
    const int64_t nblk = (int64_t)nba * nbb;
    int64_t *cnt = (int64_t *)calloc((size_t)nblk, sizeof(int64_t));
    for (int64_t q = 0; q < 3 * nblk; ++q) R[q] = 0.0;
    for (int64_t i = 0; i < s->N; ++i) {
        int qa, qb;
        block_of(s, i, B, &qa, &qb);
        const int64_t q = (int64_t)qb * nba + qa;
        for (int k = 0; k < 3; ++k) R[3 * q + k] += s->pos[k * s->N + i];
        cnt[q]++;
    }
    for (int64_t q = 0; q < nblk; ++q)
        for (int k = 0; k < 3; ++k) R[3 * q + k] /= (double)cnt[q];
    free(cnt);
}

void ora_ddr_moments(const ora_system *s, const double *n, int B, double *feat) {
    const int nba = s->geo.n_cells[0] / B, nbb = s->geo.n_cells[1] / B;
    const int64_t nblk = (int64_t)nba * nbb, N = s->N;
    double *R = (double *)malloc(sizeof(double) * 3 * (size_t)nblk);
    block_centroids(s, B, R);
    for (int64_t q = 0; q < 12 * nblk; ++q) feat[q] = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        int qa, qb;
        block_of(s, i, B, &qa, &qb);
        const int64_t q = (int64_t)qb * nba + qa;
        double ni[3], d[3];
        load(n, N, i, ni);
        for (int g = 0; g < 3; ++g) d[g] = s->pos[g * N + i] - R[3 * q + g];
        for (int c = 0; c < 3; ++c) {
            feat[12 * q + c] += ni[c];
            for (int g = 0; g < 3; ++g) feat[12 * q + 3 + 3 * g + c] += d[g] * ni[c];
        }
    }
    free(R);
}

/* u += K(r) v for the vector r from the field point to the source */
static void add_dipole(const double r[3], const double v[3], double u[3]) {
    const double d = norm3(r);
    const double rh[3] = {r[0] / d, r[1] / d, r[2] / d};
    const double vr = dot3(v, rh), inv3 = 1.0 / (d * d * d);
    for (int k = 0; k < 3; ++k) u[k] += (v[k] - 3.0 * vr * rh[k]) * inv3;
}

void ora_ddr_backbone(const ora_system *s, const double *n, int B, int reach, const int64_t *sites, int64_t n_req,
                      double *u_out) {
    const int nba = s->geo.n_cells[0] / B, nbb = s->geo.n_cells[1] / B;
    const int64_t nblk = (int64_t)nba * nbb, N = s->N;
    double *R = (double *)malloc(sizeof(double) * 3 * (size_t)nblk);
    double *feat = (double *)malloc(sizeof(double) * 12 * (size_t)nblk);
    block_centroids(s, B, R);
    ora_ddr_moments(s, n, B, feat);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < n_req; ++t) {
        const int64_t i = sites[t];
        int qa, qb;
        block_of(s, i, B, &qa, &qb);
        double pi[3], u[3] = {0.0, 0.0, 0.0};
        load(s->pos, N, i, pi);
        /* near: every site of the blocks within reach */
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            int ja, jb;
            block_of(s, j, B, &ja, &jb);
            if (abs(ja - qa) > reach || abs(jb - qb) > reach) continue;
            double r[3], nj[3];
            load(s->pos, N, j, r);
            for (int k = 0; k < 3; ++k) r[k] -= pi[k];
            load(n, N, j, nj);
            add_dipole(r, nj, u);
        }
        /* far: one dipole per block */
        for (int ob = 0; ob < nbb; ++ob)
            for (int oa = 0; oa < nba; ++oa) {
                if (abs(oa - qa) <= reach && abs(ob - qb) <= reach) continue;
                const int64_t q = (int64_t)ob * nba + oa;
                double r[3];
                for (int k = 0; k < 3; ++k) r[k] = R[3 * q + k] - pi[k];
                add_dipole(r, &feat[12 * q], u);
            }
        for (int k = 0; k < 3; ++k) u_out[3 * t + k] = u[k];
    }
    free(R);
    free(feat);
}

/* Least squares per block: r_i ~ c0 + (r_i - R_b) . c1 over the block's
 * sites, component by component (normal equations of the 4 unknowns,
 * Gaussian elimination with partial pivoting). */
void ora_ddr_project(const ora_system *s, const double *r, int B, double *coef) {
    const int nba = s->geo.n_cells[0] / B, nbb = s->geo.n_cells[1] / B;
    const int64_t nblk = (int64_t)nba * nbb, N = s->N;
    double *R = (double *)malloc(sizeof(double) * 3 * (size_t)nblk);
    double *A = (double *)calloc((size_t)nblk * 16, sizeof(double));
    double *y = (double *)calloc((size_t)nblk * 12, sizeof(double));
    block_centroids(s, B, R);
    for (int64_t i = 0; i < N; ++i) {
        int qa, qb;
        block_of(s, i, B, &qa, &qb);
        const int64_t q = (int64_t)qb * nba + qa;
        double x[4] = {1.0, 0.0, 0.0, 0.0};
        for (int g = 0; g < 3; ++g) x[1 + g] = s->pos[g * N + i] - R[3 * q + g];
        for (int a = 0; a < 4; ++a) {
            for (int b = 0; b < 4; ++b) A[16 * q + 4 * a + b] += x[a] * x[b];
            for (int c = 0; c < 3; ++c) y[12 * q + 3 * a + c] += x[a] * r[c * N + i];
        }
    }
    for (int64_t q = 0; q < nblk; ++q) {
        double M[4][7];
        for (int a = 0; a < 4; ++a) {
            for (int b = 0; b < 4; ++b) M[a][b] = A[16 * q + 4 * a + b];
            for (int c = 0; c < 3; ++c) M[a][4 + c] = y[12 * q + 3 * a + c];
        }
        for (int col = 0; col < 4; ++col) {
            int piv = col;
            for (int a = col + 1; a < 4; ++a)
                if (fabs(M[a][col]) > fabs(M[piv][col])) piv = a;
            for (int b = 0; b < 7; ++b) {
                const double t = M[col][b];
                M[col][b] = M[piv][b];
                M[piv][b] = t;
            }
            for (int a = 0; a < 4; ++a) {
                if (a == col) continue;
                const double f = M[a][col] / M[col][col];
                for (int b = col; b < 7; ++b) M[a][b] -= f * M[col][b];
            }
        }
        /* unknowns: row 0 -> c0, rows 1..3 -> c1[g] */
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) coef[12 * q + 3 * a + c] = M[a][4 + c] / M[a][a];
    }
    free(R);
    free(A);
    free(y);
}

void ora_ddr_expand(const ora_system *s, const double *coef, int B, double *r) {
    const int nba = s->geo.n_cells[0] / B, nbb = s->geo.n_cells[1] / B;
    const int64_t nblk = (int64_t)nba * nbb, N = s->N;
    double *R = (double *)malloc(sizeof(double) * 3 * (size_t)nblk);
    block_centroids(s, B, R);
    for (int64_t i = 0; i < N; ++i) {
        int qa, qb;
        block_of(s, i, B, &qa, &qb);
        const int64_t q = (int64_t)qb * nba + qa;
        for (int c = 0; c < 3; ++c) {
            double v = coef[12 * q + c];
            for (int g = 0; g < 3; ++g) v += (s->pos[g * N + i] - R[3 * q + g]) * coef[12 * q + 3 + 3 * g + c];
            r[c * N + i] = v;
        }
    }
    free(R);
}

/* ------------------------------------------------- convolutional surrogate
 * Not in the paper: a learned stand-in for the dipolar field.  Plain loops
 * over the definitions of a zero-padded 3x3 cross-correlation, SiLU, and the
 * Adam update. */

/* When non-zero the conv layers skip the bfloat16 rounding of their
 * operands (exact arithmetic), for finite-difference checks of the chain rule. */
static int g_conv_exact = 0;
void ora_conv_set_exact(int on) { g_conv_exact = on; }

static double q16(double x);

/* Round to bfloat16, nearest-even (8 significant bits). */
double ora_bf16(double x) {
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    double m = frexp(x, &e);          /* x = m 2^e, 0.5 <= |m| < 1 */
    double s = ldexp(m, 8);           /* 8 significant bits -> integer part */
    double r = nearbyint(s);          /* default rounding mode: ties to even */
    return ldexp(r, e - 8);
}

static double q16(double x) { return g_conv_exact ? x : ora_bf16(x); }

void ora_conv3x3_fwd(int B, int H, int W, int Cin, int Cout, const double *x, const double *w,
                     const double *bias, double *z) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; ++b)
        for (int y = 0; y < H; ++y)
            for (int xx = 0; xx < W; ++xx)
                for (int co = 0; co < Cout; ++co) {
                    double acc = bias[co];
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int sy = y + ky - 1, sx = xx + kx - 1;
                            if (sy < 0 || sy >= H || sx < 0 || sx >= W) continue;
                            for (int ci = 0; ci < Cin; ++ci)
                                acc += q16(x[(((int64_t)b * H + sy) * W + sx) * Cin + ci]) *
                                       q16(w[((ky * 3 + kx) * Cin + ci) * Cout + co]);
                        }
                    z[(((int64_t)b * H + y) * W + xx) * Cout + co] = acc;
                }
}

/* Chain rule of the forward definition:
 *   dL/dx[b,sy,sx,ci] = sum over (y,x,ky,kx,co) with sy = y+ky-1, sx = x+kx-1 of dz[b,y,x,co] w[ky,kx,ci,co]
 *   dL/dw[ky,kx,ci,co] = sum over (b,y,x) of x[b,y+ky-1,x+kx-1,ci] dz[b,y,x,co]
 *   dL/db[co]          = sum over (b,y,x) of dz[b,y,x,co] */
void ora_conv3x3_bwd(int B, int H, int W, int Cin, int Cout, const double *x, const double *w,
                     const double *dz, double *dx, double *dw, double *db) {
    if (dx) {
#pragma omp parallel for collapse(2) schedule(static)
        for (int b = 0; b < B; ++b)
            for (int sy = 0; sy < H; ++sy)
                for (int sx = 0; sx < W; ++sx)
                    for (int ci = 0; ci < Cin; ++ci) {
                        double acc = 0.0;
                        for (int ky = 0; ky < 3; ++ky)
                            for (int kx = 0; kx < 3; ++kx) {
                                int y = sy - ky + 1, xx = sx - kx + 1;
                                if (y < 0 || y >= H || xx < 0 || xx >= W) continue;
                                for (int co = 0; co < Cout; ++co)
                                    acc += q16(dz[(((int64_t)b * H + y) * W + xx) * Cout + co]) *
                                           q16(w[((ky * 3 + kx) * Cin + ci) * Cout + co]);
                            }
                        dx[(((int64_t)b * H + sy) * W + sx) * Cin + ci] = acc;
                    }
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < 9; ++k)
        for (int ci = 0; ci < Cin; ++ci)
            for (int co = 0; co < Cout; ++co) {
                int ky = k / 3, kx = k % 3;
                double acc = 0.0;
                for (int b = 0; b < B; ++b)
                    for (int y = 0; y < H; ++y)
                        for (int xx = 0; xx < W; ++xx) {
                            int sy = y + ky - 1, sx = xx + kx - 1;
                            if (sy < 0 || sy >= H || sx < 0 || sx >= W) continue;
                            acc += q16(x[(((int64_t)b * H + sy) * W + sx) * Cin + ci]) *
                                   q16(dz[(((int64_t)b * H + y) * W + xx) * Cout + co]);
                        }
                dw[(k * Cin + ci) * Cout + co] = acc;
            }
    for (int co = 0; co < Cout; ++co) {
        double acc = 0.0;
        for (int64_t q = 0; q < (int64_t)B * H * W; ++q) acc += dz[q * Cout + co];
        db[co] = acc;
    }
}

void ora_silu(int64_t n, const double *z, double *y, double *dydz) {
    for (int64_t k = 0; k < n; ++k) {
        double s = 1.0 / (1.0 + exp(-z[k]));
        if (y) y[k] = z[k] * s;
        if (dydz) dydz[k] = s * (1.0 + z[k] * (1.0 - s));
    }
}

void ora_adam(int64_t n, double *p, double *m, double *v, const double *g, double lr, double b1, double b2,
              double eps, int t) {
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int64_t k = 0; k < n; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        double mh = m[k] / c1, vh = v[k] / c2;
        p[k] -= lr * mh / (sqrt(vh) + eps);
    }
}

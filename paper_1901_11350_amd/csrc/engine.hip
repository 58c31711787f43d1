// engine.hip -- host side of the MI355X atomistic-spin engine: state,
// neighbour-shell bond tables, buffer management, kernel launches and the
// C ABI declared in include/sp_engine.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <mutex>
#include <set>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "sp_engine.h"
#include "kernels_field.hpp"
#include "kernels_reduce.hpp"
#include "kernels_dipole.hpp"
#include "kernels_fused2d.hpp"
#include "kernels_tile.hpp"
#include "kernels_gneb.hpp"
#include "kernels_conv.hpp"
#include "kernels_ddr.hpp"
#include "kernels_fft.hpp"
#include "kernels_mc.hpp"
#include "kernels_fused3d.hpp"
#include "kernels_persist2d.hpp"
#include "kernels_stencil.hpp"

namespace {

// CODATA 2018 (SI) in meV / Tesla / ps / Angstrom.
constexpr double kJperMeV = 1.602176634e-22;
constexpr double kMuB = 9.2740100783e-24 / kJperMeV;            // meV/T
constexpr double kKB = 1.380649e-23 / kJperMeV;                 // meV/K
constexpr double kGamma = 0.176085963023;                       // rad/(ps T)
constexpr double kCdd = 1.00000000055e-7 * 9.2740100783e-24 * 9.2740100783e-24 / 1e-30 / kJperMeV;  // meV

struct HostGeo {
    double bravais[9];
    int nb;
    double basis[3 * SP_MAX_BASIS];
    int n[3];
    int per[3];
    double a;
};

struct HostHam {
    double mu[SP_MAX_BASIS];
    double B[3];
    double K[SP_MAX_BASIS];
    double Kax[3 * SP_MAX_BASIS];
    int n_exch, n_dmi;
    double J[SP_MAX_SHELLS], D[SP_MAX_SHELLS];
    int dmi_kind;
    int ddi;
    int n_gauss;
    double ga[SP_MAX_GAUSS], gsigma[SP_MAX_GAUSS], gc[3 * SP_MAX_GAUSS];   // centres normalised
};

struct HostBond {
    int bi, bj, d[3], shell;
    double J, D[3];
};

const char* kVersion = "sp_engine 0.1 (gfx950)";

}  // namespace

struct SurrogateState;
void surrogate_free(SurrogateState* s);
struct FftState;
void fft_free(FftState* s);

// One captured chunk of sp_run: `steps` step launches (+ an observation),
// valid for the parameters, buffers and step path it was captured with.
struct RunGraph {
    sp_llg_params p;
    int steps;
    bool observe;
    double tol;
    const void* n_first;     // the buffer the chunk starts from
    const void* n_other;
    const double* obs;       // the run's observation array at capture
    long long obs_cap;
    std::string path;
    hipGraphExec_t exec;
};

struct sp_engine {
    int device = 0;
    int precision = SP_F32;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    bool has_geo = false, has_ham = false, has_spins = false;
    HostGeo geo{};
    HostHam ham{};
    std::vector<HostBond> bonds;
    std::vector<int> bstart;
    int N = 0;
    int R = 0;            // stencil reach in cells (max |d| over bonds)
    bool planar = true;   // every bond has dc == 0
    uint64_t step = 0;
    const char* path = "none";
    bool fused_ok = false;
    bool tile_ok = false;   // the fused tile path takes this lattice (basis, or 3D without a stencil)
    std::vector<HostBond> all_bonds;  // every bond of the requested shells (zero ones included)
    int n_shells = 0;
    int shape = -1;                   // sp::Shape2D matched by the bond table, or -1
    int shape_ndmi = 0;               // 0: no DMI, 1: DMI on the first shell only
    int tile_cfg = 0;                 // index into the shape-path tile configurations
    int shape3 = -1;                  // sp::Shape3D matched by a 3D one-atom bond table, or -1
    bool explicit_pairs = false;      // bond table from sp_set_pairs (no compile-time stencil paths)
    int shape3_ndmi = 0;              // DMI on the first shell
    int shape3_dk = 0;                // sp::Dmi3 of the streamed step kernel
    int tile3_cfg = 0;                // index into the 3D tile configurations
    int persist_cfg = 0;              // index into the persistent-path tile configurations
    std::vector<unsigned char> mc_col;  // Metropolis colour of each (cell class, atom)
    int mc_m[3] = {1, 1, 1};            // periods of the colouring
    int mc_ncol = 0;
    std::string path_label;

    size_t esz() const { return precision == SP_F64 ? 8 : 4; }

    // device buffers (engine precision unless noted)
    void* d_n = nullptr;
    void* d_n2 = nullptr;
    void* d_np = nullptr;
    void* d_A = nullptr;
    void* d_g = nullptr;
    void* d_gdd = nullptr;
    void* d_gddp = nullptr;
    void* d_pos = nullptr;
    void* d_ddpart = nullptr;
    int dd_slices = 1;
    int4* d_bond = nullptr;
    int* d_bstart = nullptr;
    void* d_J = nullptr;
    void* d_D = nullptr;
    void* d_J64 = nullptr;              // FP64 copies for an FP32 engine's Monte Carlo decisions
    void* d_D64 = nullptr;
    double* d_partials = nullptr;     // observe stage-1 rows
    int partial_rows = 0;
    double* d_obs = nullptr;          // observations of a run, OBS_NVALS each
    int64_t obs_cap = 0;
    int* d_flag = nullptr;            // abort flag (non-finite torque)
    long long* d_abort_step = nullptr;
    uint32_t* d_pflags = nullptr;     // persistent path: one flag line per tile
    int pflag_tiles = 0;
    uint32_t pgen = 0;                // every flag is <= pgen between launches
    int* d_pstatus = nullptr;         // persistent path: nonzero after a failed wait
    double* h_pin = nullptr;          // pinned staging for small results
    // replayed step graphs (sp_run): device step counter + observation index,
    // a staging row for the chunk's observation, and the cached executables
    unsigned long long* d_step = nullptr;
    long long* d_obs_index = nullptr;
    double* d_obs_stage = nullptr;
    const unsigned long long* cap_step_dev = nullptr;   // set while capturing
    unsigned int cap_step_off = 0;
    bool graphs_on = true;
    std::vector<RunGraph> graphs;
    SurrogateState* sur = nullptr;    // learned dipole field (sp_ddi_*)
    FftState* fft = nullptr;          // FFT-convolution dipole field (SP_DDI_FFT)
};

namespace {

int fail(sp_engine* e, int code, const std::string& msg) {
    if (e) e->err = msg;
    return code;
}

#define HIPCHK(e, call)                                                                       \
    do {                                                                                      \
        hipError_t _s = (call);                                                               \
        if (_s != hipSuccess)                                                                 \
            return fail((e), SP_E_HIP, std::string(#call) + ": " + hipGetErrorString(_s));    \
    } while (0)

void dfree(void*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <typename P>
int dalloc(sp_engine* e, P*& p, size_t bytes) {
    if (p) {
        (void)hipFree(p);
        p = nullptr;
    }
    if (bytes == 0) return SP_OK;
    void* q = nullptr;
    hipError_t s = hipMalloc(&q, bytes);
    if (s != hipSuccess) {
        (void)hipGetLastError();
        return fail(e, SP_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    p = static_cast<P*>(q);
    return SP_OK;
}

void drop_graphs(sp_engine* e) {
    for (RunGraph& g : e->graphs) (void)hipGraphExecDestroy(g.exec);
    e->graphs.clear();
}

void free_state_buffers(sp_engine* e) {
    drop_graphs(e);
    dfree(e->d_n); dfree(e->d_n2); dfree(e->d_np); dfree(e->d_A); dfree(e->d_g);
    dfree(e->d_gdd); dfree(e->d_gddp); dfree(e->d_pos); dfree(e->d_ddpart);
    void* p = e->d_bond; dfree(p); e->d_bond = nullptr;
    p = e->d_bstart; dfree(p); e->d_bstart = nullptr;
    dfree(e->d_J); dfree(e->d_D); dfree(e->d_J64); dfree(e->d_D64);
    fft_free(e->fft);
    e->fft = nullptr;
}

// ------------------------------------------------------------ bond table
// Neighbour shells per basis atom: candidates within +-4 cells (axes with a
// single open cell carry no translation) sorted by distance; distances within
// 1e-6 lattice constants form one shell.  Bonds of the first
// max(n_exch, n_dmi) shells are kept in both directions.
int build_bonds(sp_engine* e, const HostGeo& g, const HostHam& h, std::vector<HostBond>& out,
                std::vector<int>& start, std::vector<HostBond>& all) {
    struct Cand {
        int bj, d[3];
        double dist, r[3];
    };
    out.clear();
    all.clear();
    start.assign(g.nb + 1, 0);
    const int want = std::max(h.n_exch, h.n_dmi);
    int ext[3];
    for (int k = 0; k < 3; ++k) ext[k] = (g.n[k] > 1 || g.per[k]) ? 4 : 0;
    for (int bi = 0; bi < g.nb; ++bi) {
        start[bi] = (int)out.size();
        if (want == 0) continue;
        std::vector<Cand> cs;
        for (int bj = 0; bj < g.nb; ++bj)
            for (int x = -ext[0]; x <= ext[0]; ++x)
                for (int y = -ext[1]; y <= ext[1]; ++y)
                    for (int z = -ext[2]; z <= ext[2]; ++z) {
                        Cand c{bj, {x, y, z}, 0.0, {0, 0, 0}};
                        for (int k = 0; k < 3; ++k)
                            c.r[k] = x * g.bravais[k] + y * g.bravais[3 + k] + z * g.bravais[6 + k] +
                                     g.basis[3 * bj + k] - g.basis[3 * bi + k];
                        c.dist = std::sqrt(c.r[0] * c.r[0] + c.r[1] * c.r[1] + c.r[2] * c.r[2]);
                        if (c.dist >= 1e-6) cs.push_back(c);
                    }
        std::stable_sort(cs.begin(), cs.end(), [](const Cand& a, const Cand& b) { return a.dist < b.dist; });
        int shell = -1;
        double shell_d = 0.0;
        for (const Cand& c : cs) {
            if (shell < 0 || c.dist > shell_d + 1e-6) {
                ++shell;
                shell_d = c.dist;
            }
            if (shell >= want) break;
            HostBond b{};
            b.bi = bi;
            b.bj = c.bj;
            for (int k = 0; k < 3; ++k) b.d[k] = c.d[k];
            b.shell = shell;
            b.J = shell < h.n_exch ? h.J[shell] : 0.0;
            const double Dm = shell < h.n_dmi ? h.D[shell] : 0.0;
            const double ux = c.r[0] / c.dist, uy = c.r[1] / c.dist, uz = c.r[2] / c.dist;
            if (h.dmi_kind == SP_DMI_BULK) {
                b.D[0] = Dm * ux; b.D[1] = Dm * uy; b.D[2] = Dm * uz;
            } else {  // z x r_hat
                b.D[0] = -Dm * uy; b.D[1] = Dm * ux; b.D[2] = 0.0;
            }
            all.push_back(b);
            if (b.J == 0.0 && b.D[0] == 0.0 && b.D[1] == 0.0 && b.D[2] == 0.0) continue;
            out.push_back(b);
        }
        if (shell + 1 < want)
            return fail(e, SP_E_ARG, "basis atom " + std::to_string(bi) + " has only " + std::to_string(shell + 1) +
                                         " neighbour shells within 4 cells; " + std::to_string(want) + " requested");
    }
    start[g.nb] = (int)out.size();
    return SP_OK;
}

// ------------------------------------------------------- kernel arguments
template <typename T>
sp::Phys<T> make_phys(const sp_engine* e, const sp_llg_params* p) {
    sp::Phys<T> P{};
    P.nb = e->geo.nb;
    for (int b = 0; b < e->geo.nb; ++b) {
        const double mm = e->ham.mu[b] * kMuB;
        P.mumuB[b] = (T)mm;
        for (int k = 0; k < 3; ++k) {
            P.gZ[b][k] = (T)(-mm * e->ham.B[k]);
            P.Kax[b][k] = (T)e->ham.Kax[3 * b + k];
        }
        P.K2[b] = (T)(2.0 * e->ham.K[b]);
        P.sigma[b] = T(0);
        if (p && p->T_K > 0.0)
            P.sigma[b] = (T)std::sqrt(2.0 * p->alpha * kKB * p->T_K / (kGamma * mm * p->dt_ps));
    }
    P.ng = e->ham.n_gauss;
    for (int k = 0; k < P.ng; ++k) {
        P.ga[k] = (T)e->ham.ga[k];
        P.gis2[k] = (T)(1.0 / (e->ham.gsigma[k] * e->ham.gsigma[k]));
        for (int q = 0; q < 3; ++q) P.gc[k][q] = (T)e->ham.gc[3 * k + q];
    }
    return P;
}

template <typename T>
sp::LLGArgs<T> make_llg(const sp_llg_params* p, uint64_t step, uint32_t replica) {
    sp::LLGArgs<T> A{};
    A.gp = (T)(kGamma / (1.0 + p->alpha * p->alpha));
    A.alpha = (T)p->alpha;
    A.dt = (T)p->dt_ps;
    A.thermal = p->T_K > 0.0 ? 1 : 0;
    A.key.seed_lo = (uint32_t)p->seed;
    A.key.seed_hi = (uint32_t)(p->seed >> 32);
    A.key.step_lo = (uint32_t)step;
    A.key.step_hi = (uint32_t)(step >> 32);
    A.key.replica = replica;
    return A;
}

// LLG arguments of a step launch of the engine: while a step graph is being
// captured, the launch reads its Philox step from the device counter.
template <typename T>
sp::LLGArgs<T> make_step_llg(const sp_engine* e, const sp_llg_params* p, uint64_t step) {
    sp::LLGArgs<T> A = make_llg<T>(p, step, p->replica);
    if (e->cap_step_dev) {
        A.step_dev = e->cap_step_dev;
        A.step_off = e->cap_step_off;
    }
    return A;
}

sp::Lattice make_lattice(const sp_engine* e) {
    sp::Lattice L{};
    for (int k = 0; k < 3; ++k) {
        L.n[k] = e->geo.n[k];
        L.per[k] = e->geo.per[k];
    }
    L.nb = e->geo.nb;
    L.N = e->N;
    L.bond = e->d_bond;
    L.bstart = e->d_bstart;
    return L;
}

template <typename T>
sp::BondCoef<T> make_coef(const sp_engine* e) {
    return sp::BondCoef<T>{static_cast<const T*>(e->d_J), static_cast<const T*>(e->d_D)};
}

// FP64 couplings for every engine precision (an FP32 engine keeps FP64
// copies for its FP64 decisions).
sp::BondCoef<double> make_coef64(const sp_engine* e) {
    return sp::BondCoef<double>{static_cast<const double*>(e->precision == SP_F64 ? e->d_J : e->d_J64),
                                static_cast<const double*>(e->precision == SP_F64 ? e->d_D : e->d_D64)};
}

inline unsigned blocks_for(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// ----------------------------------------------------------------- dipole
template <typename T>
int launch_direct_sum(sp_engine* e, const void* n, void* gdd, const int* gate = nullptr) {
    sp::DipoleArgs<T> a{};
    a.N = e->N;
    a.cells = e->geo.n[0] * e->geo.n[1] * e->geo.n[2];
    a.slices = e->dd_slices;
    const int tiles = (e->N + 255) / 256;
    a.slice_len = ((tiles + a.slices - 1) / a.slices) * 256;
    for (int b = 0; b < e->geo.nb; ++b) a.mu[b] = (T)e->ham.mu[b];
    constexpr int IPT = 2;
    dim3 grid((unsigned)((e->N + 256 * IPT - 1) / (256 * IPT)), (unsigned)a.slices);
    hipLaunchKernelGGL((sp::k_dipole_partial<T, IPT>), grid, dim3(256), 0, e->stream, a,
                       static_cast<const T*>(e->d_pos), static_cast<const T*>(n), static_cast<T*>(e->d_ddpart), gate);
    hipLaunchKernelGGL((sp::k_dipole_finish<T>), dim3(blocks_for(3LL * e->N)), dim3(256), 0, e->stream, a,
                       (T)kCdd, static_cast<const T*>(e->d_ddpart), static_cast<T*>(gdd), gate);
    HIPCHK(e, hipGetLastError());
    return SP_OK;
}

// Scratch of sp_dipole_gradient_dev_noalloc: the S slices of partial sums
// of the direct sum live in this file-scope device array instead of engine
// memory.  Every GPU the library runs on holds its own copy until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
bool g_scratch_tried[kScratchDevices] = {};

// Looks the array up once per device, with that device current (sp_create
// calls it after hipSetDevice).  Returns the device address or nullptr.
void* scratch_for_device(int device) {
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_tried[device]) {
        void* ptr = nullptr;
        const hipError_t st = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[device] = st == hipSuccess ? ptr : nullptr;
        g_scratch_tried[device] = true;
        if (st != hipSuccess) (void)hipGetLastError();
    }
    return g_scratch_ptr[device];
}

// The direct sum with its partials in `part` (the engine's buffer or the
// static scratch); the partial kernel writes every element of the
// slices * 3N values before the finish kernel reads them.
template <typename T>
int launch_direct_sum_into(sp_engine* e, const void* n, void* gdd, void* part) {
    sp::DipoleArgs<T> a{};
    a.N = e->N;
    a.cells = e->geo.n[0] * e->geo.n[1] * e->geo.n[2];
    a.slices = e->dd_slices;
    const int tiles = (e->N + 255) / 256;
    a.slice_len = ((tiles + a.slices - 1) / a.slices) * 256;
    for (int b = 0; b < e->geo.nb; ++b) a.mu[b] = (T)e->ham.mu[b];
    constexpr int IPT = 2;
    dim3 grid((unsigned)((e->N + 256 * IPT - 1) / (256 * IPT)), (unsigned)a.slices);
    hipLaunchKernelGGL((sp::k_dipole_partial<T, IPT>), grid, dim3(256), 0, e->stream, a,
                       static_cast<const T*>(e->d_pos), static_cast<const T*>(n), static_cast<T*>(part), nullptr);
    hipLaunchKernelGGL((sp::k_dipole_finish<T>), dim3(blocks_for(3LL * e->N)), dim3(256), 0, e->stream, a,
                       (T)kCdd, static_cast<const T*>(part), static_cast<T*>(gdd), nullptr);
    HIPCHK(e, hipGetLastError());
    return SP_OK;
}

template <typename T>
int surrogate_field(sp_engine* e, const void* n, void* gdd);
template <typename T>
int fft_field(sp_engine* e, const void* n, void* gdd);
template <typename T>
int fft_setup(sp_engine* e);
int fft_check(sp_engine* e);

// Dipole gradient for the step/gradient/observe paths: the direct sum, the
// FFT convolution, or the learned surrogate with its residual check and
// direct-sum fallback.
template <typename T>
int launch_dipole(sp_engine* e, const void* n, void* gdd) {
    if (e->ham.ddi == SP_DDI_SURROGATE) return surrogate_field<T>(e, n, gdd);
    if (e->ham.ddi == SP_DDI_FFT) return fft_field<T>(e, n, gdd);
    return launch_direct_sum<T>(e, n, gdd);
}

// --------------------------------------------------------------- observe
template <typename T>
sp::Site2D<T> make_site2d(const sp_engine* e, const sp_llg_params* p);
template <typename T, int S>
sp::ShapeCoef<T> shape_coef_for(const sp_engine* e);
template <typename T, int S>
sp::ShapeCoef3<T> shape_coef3_for(const sp_engine* e);

// Observables on the stencil path's tiles (64 x 16, four sites per thread):
// one partial row per workgroup, at most partial_rows workgroups.  Returns
// the number of rows.
template <typename T, int S>
int go_observe_shape(sp_engine* e, const void* n) {
    constexpr int TX = 64, TY = 16, NT = 256;   // 1024 threads measured slower
    sp::TileMap M{};
    M.tiles_x = (e->geo.n[0] + TX - 1) / TX;
    M.tiles_y = (e->geo.n[1] + TY - 1) / TY;
    const int rows = std::min(M.tiles_x * M.tiles_y, e->partial_rows);
    const sp::ShapeCoef<T> C = shape_coef_for<T, S>(e);
    const sp::Site2D<T> Q = make_site2d<T>(e, nullptr);
    if (e->shape_ndmi)
        hipLaunchKernelGGL((sp::k_observe_shape<T, S, sp::ShapeTab<S>::NB0, TX, TY, NT>), dim3((unsigned)rows),
                           dim3(NT), 0, e->stream, C, Q, M, static_cast<const T*>(n), e->d_partials);
    else
        hipLaunchKernelGGL((sp::k_observe_shape<T, S, 0, TX, TY, NT>), dim3((unsigned)rows), dim3(NT), 0, e->stream,
                           C, Q, M, static_cast<const T*>(n), e->d_partials);
    return rows;
}

// The same on the streamed 3D path's lattices: 32 x 8 tiles of one plane
// (with the planes either side) per work item.
template <typename T, int S>
int go_observe_shape3(sp_engine* e, const void* n) {
    constexpr int TX = 32, TY = 8;
    const int tiles_x = (e->geo.n[0] + TX - 1) / TX, tiles_y = (e->geo.n[1] + TY - 1) / TY;
    const long long items = (long long)tiles_x * tiles_y * e->geo.n[2];
    const int rows = (int)std::min<long long>(items, e->partial_rows);
    const sp::ShapeCoef3<T> C = shape_coef3_for<T, S>(e);
    const sp::Site2D<T> Q = make_site2d<T>(e, nullptr);
    if (e->shape3_ndmi)
        hipLaunchKernelGGL((sp::k_observe_shape3<T, S, sp::ShapeTab3<S>::NB0, TX, TY>), dim3((unsigned)rows),
                           dim3(TX * TY), 0, e->stream, C, Q, e->geo.n[2], e->geo.per[2], tiles_x, tiles_y,
                           static_cast<const T*>(n), e->d_partials);
    else
        hipLaunchKernelGGL((sp::k_observe_shape3<T, S, 0, TX, TY>), dim3((unsigned)rows), dim3(TX * TY), 0, e->stream,
                           C, Q, e->geo.n[2], e->geo.per[2], tiles_x, tiles_y, static_cast<const T*>(n), e->d_partials);
    return rows;
}

template <typename T>
int launch_observe(sp_engine* e, const void* n, double* out, long long step, bool with_flag,
                   const unsigned long long* step_dev = nullptr, int step_off = 0, double tol = 0.0) {
    if (e->shape3 >= 0 && !e->ham.ddi && e->ham.n_gauss == 0) {
        int rows;
        switch (e->shape3) {
            case sp::SH3_SC1: rows = go_observe_shape3<T, sp::SH3_SC1>(e, n); break;
            case sp::SH3_SC2: rows = go_observe_shape3<T, sp::SH3_SC2>(e, n); break;
            default: rows = go_observe_shape3<T, sp::SH3_SC3>(e, n); break;
        }
        hipLaunchKernelGGL(sp::k_observe_final, dim3(1), dim3(256), 0, e->stream, e->d_partials, rows, out,
                           with_flag ? e->d_flag : nullptr, e->d_abort_step, step, step_dev, step_off, tol);
        HIPCHK(e, hipGetLastError());
        return SP_OK;
    }
    if (e->shape >= 0 && !e->ham.ddi && e->ham.n_gauss == 0) {
        int rows;
        switch (e->shape) {
            case sp::SH_SQ1: rows = go_observe_shape<T, sp::SH_SQ1>(e, n); break;
            case sp::SH_SQ2: rows = go_observe_shape<T, sp::SH_SQ2>(e, n); break;
            case sp::SH_SQ3: rows = go_observe_shape<T, sp::SH_SQ3>(e, n); break;
            case sp::SH_TRI1: rows = go_observe_shape<T, sp::SH_TRI1>(e, n); break;
            case sp::SH_TRI2: rows = go_observe_shape<T, sp::SH_TRI2>(e, n); break;
            default: rows = go_observe_shape<T, sp::SH_TRI3>(e, n); break;
        }
        hipLaunchKernelGGL(sp::k_observe_final, dim3(1), dim3(256), 0, e->stream, e->d_partials, rows, out,
                           with_flag ? e->d_flag : nullptr, e->d_abort_step, step, step_dev, step_off, tol);
        HIPCHK(e, hipGetLastError());
        return SP_OK;
    }
    const void* gdd = nullptr;
    if (e->ham.ddi) {
        int rc = launch_dipole<T>(e, n, e->d_gdd);
        if (rc) return rc;
        gdd = e->d_gdd;
    }
    const sp::Phys<T> P = make_phys<T>(e, nullptr);
    hipLaunchKernelGGL((sp::k_observe_partial<T>), dim3(e->partial_rows), dim3(256), 0, e->stream,
                       make_lattice(e), make_coef<T>(e), P, static_cast<const T*>(n), static_cast<const T*>(gdd),
                       e->d_partials);
    hipLaunchKernelGGL(sp::k_observe_final, dim3(1), dim3(256), 0, e->stream, e->d_partials, e->partial_rows, out,
                       with_flag ? e->d_flag : nullptr, e->d_abort_step, step, step_dev, step_off, tol);
    HIPCHK(e, hipGetLastError());
    return SP_OK;
}

void obs_from(const double* v, int64_t step, int N, sp_observation* o) {
    o->step = step;
    o->per_term[0] = v[sp::OBS_EZ];
    o->per_term[1] = v[sp::OBS_EK];
    o->per_term[2] = v[sp::OBS_EJ];
    o->per_term[3] = v[sp::OBS_ED];
    o->per_term[4] = v[sp::OBS_EDD];
    o->E = o->per_term[0] + o->per_term[1] + o->per_term[2] + o->per_term[3] + o->per_term[4];
    o->max_torque = v[sp::OBS_NONFINITE] > 0.0 ? NAN : v[sp::OBS_TMAX];
    o->M[0] = v[sp::OBS_MX] / N;
    o->M[1] = v[sp::OBS_MY] / N;
    o->M[2] = v[sp::OBS_MZ] / N;
    o->max_norm_dev = v[sp::OBS_NDEV];
}

// ------------------------------------------------------------ LLG step
template <typename T>
sp::Stencil2D<T> make_stencil2d(const sp_engine* e) {
    sp::Stencil2D<T> S{};
    S.nbond = (int)e->bonds.size();
    for (int q = 0; q < S.nbond; ++q) {
        const HostBond& b = e->bonds[q];
        S.da[q] = b.d[0];
        S.db[q] = b.d[1];
        S.J[q] = (T)b.J;
        for (int k = 0; k < 3; ++k) S.D[q][k] = (T)b.D[k];
    }
    return S;
}

template <typename T>
sp::Site2D<T> make_site2d(const sp_engine* e, const sp_llg_params* p) {
    const sp::Phys<T> P = make_phys<T>(e, p);
    sp::Site2D<T> Q{};
    Q.na = e->geo.n[0];
    Q.nb = e->geo.n[1];
    Q.per_a = e->geo.per[0];
    Q.per_b = e->geo.per[1];
    Q.mumuB = P.mumuB[0];
    Q.inv_mumuB = (T)(1.0 / (e->ham.mu[0] * kMuB));
    for (int k = 0; k < 3; ++k) {
        Q.gZ[k] = P.gZ[0][k];
        Q.Kax[k] = P.Kax[0][k];
    }
    Q.K2 = P.K2[0];
    Q.sigma = P.sigma[0];
    return Q;
}

template <typename T, int TX, int TY, int R>
void launch_fused2d(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    dim3 grid((unsigned)((e->geo.n[0] + TX - 1) / TX), (unsigned)((e->geo.n[1] + TY - 1) / TY));
    hipLaunchKernelGGL((sp::k_depondt_fused2d<T, TX, TY, R>), grid, dim3(256), 0, e->stream, make_stencil2d<T>(e),
                       make_site2d<T>(e, p), make_step_llg<T>(e, p, step), e->d_flag, static_cast<const T*>(nin),
                       static_cast<T*>(nout));
}

// ------------------------------------------------ fused tile path (basis)
// Lattices with a basis, or 3D bond tables without a compile-time stencil.
// One thread per owned site, so a tile holds NB x TX x TY x TZ <= 1024
// sites: 2D FP32 32 x 16 (two atoms) or 16 x 16 (three, four), FP64 16 x 16
// or 16 x 8; 3D FP32 16 x 8 x 4 (one, two atoms) or 8 x 8 x 4 (three), FP64
// 8 x 8 x 4 (one, two).  Reach up to 2 in 2D, 1 in 3D.  Every instance
// stays within the 160 KB of LDS a workgroup may hold.
int padded_bonds(const sp_engine* e);

bool tile_fits(const sp_engine* e, const HostHam& H) {
    const HostGeo& g = e->geo;
    if (H.ddi || H.n_gauss > 0 || g.nb > 4 || padded_bonds(e) > sp::kMaxStencilB) return false;
    int rc = 0;
    for (const HostBond& b : e->bonds) rc = std::max(rc, std::abs(b.d[2]));
    if (g.n[2] == 1) {
        if (g.nb == 1 || !e->planar || e->R > 2) return false;
    } else {
        if (e->R > 1 || rc > 1 || g.nb > (e->precision == SP_F64 ? 2 : 3)) return false;
        if (g.per[2] && g.n[2] <= 2) return false;
    }
    if (g.per[0] && g.n[0] <= 2 * std::max(e->R, 1)) return false;
    if (g.per[1] && g.n[1] <= 2 * std::max(e->R, 1)) return false;
    return true;
}

// Bond table of the tile kernel whose spin frame is WN x HN (x DN), block
// PN cells per atom, and predictor frame WP x HP, block PP.
// Each atom's list is padded to a multiple of four with zero bonds to the
// site's own cell (offset 0).
template <typename T>
sp::StencilB<T> make_stencilb(const sp_engine* e, int WN, int HN, int PN, int WP, int HP, int PP) {
    sp::StencilB<T> S{};
    S.nb = e->geo.nb;
    int q = 0;
    for (int beta = 0; beta < S.nb; ++beta) {
        S.bstart[beta] = q;
        for (int k = e->bstart[beta]; k < e->bstart[beta + 1]; ++k, ++q) {
            const HostBond& b = e->bonds[k];
            S.offN[q] = PN * b.bj + b.d[0] + WN * (b.d[1] + HN * b.d[2]);
            S.offP[q] = PP * b.bj + b.d[0] + WP * (b.d[1] + HP * b.d[2]);
            S.J[q] = (T)b.J;
            for (int c = 0; c < 3; ++c) S.D[q][c] = (T)b.D[c];
        }
        for (; q % 4; ++q) {   // zero bonds (the struct is value-initialised)
            S.offN[q] = 0;
            S.offP[q] = 0;
        }
    }
    S.bstart[S.nb] = q;
    return S;
}

// Bonds of the tile kernel's table once each atom's list is padded to a
// multiple of four.
int padded_bonds(const sp_engine* e) {
    int n = 0;
    for (int b = 0; b < e->geo.nb; ++b) n += (e->bstart[b + 1] - e->bstart[b] + 3) / 4 * 4;
    return n;
}

template <typename T>
sp::SiteB<T> make_siteb(const sp_engine* e, const sp_llg_params* p) {
    const sp::Phys<T> P = make_phys<T>(e, p);
    sp::SiteB<T> Q{};
    for (int k = 0; k < 3; ++k) {
        Q.n[k] = e->geo.n[k];
        Q.per[k] = e->geo.per[k];
    }
    for (int b = 0; b < e->geo.nb; ++b) {
        Q.inv_mumuB[b] = (T)(1.0 / (e->ham.mu[b] * kMuB));
        for (int k = 0; k < 3; ++k) {
            Q.gZ[b][k] = P.gZ[b][k];
            Q.Kax[b][k] = P.Kax[b][k];
        }
        Q.K2[b] = P.K2[b];
        Q.sigma[b] = P.sigma[b];
    }
    return Q;
}

template <typename T, int TX, int TY, int TZ, int R, int RC, int NB, int SOLVER>
void launch_tile_k(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    const dim3 grid((unsigned)((e->geo.n[0] + TX - 1) / TX), (unsigned)((e->geo.n[1] + TY - 1) / TY),
                    (unsigned)((e->geo.n[2] + TZ - 1) / TZ));
    constexpr int WN = TX + 4 * R, HN = TY + 4 * R, DN = TZ + 4 * RC;
    constexpr int WP = TX + 2 * R, HP = TY + 2 * R, DP = TZ + 2 * RC;
    hipLaunchKernelGGL((sp::k_fused_tile<T, TX, TY, TZ, R, RC, NB, SOLVER>), grid, dim3(NB * TX * TY * TZ), 0, e->stream,
                       make_stencilb<T>(e, WN, HN, WN * HN * DN, WP, HP, WP * HP * DP), make_siteb<T>(e, p),
                       make_step_llg<T>(e, p, step), e->d_flag,
                       static_cast<const T*>(nin), static_cast<T*>(nout));
}

template <typename T, int R, int SOLVER>
void go_tile2d(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    constexpr bool f32 = sizeof(T) == 4;
    switch (e->geo.nb) {
        case 2: launch_tile_k<T, f32 ? 32 : 16, 16, 1, R, 0, 2, SOLVER>(e, p, step, nin, nout); break;
        case 3: launch_tile_k<T, 16, f32 ? 16 : 8, 1, R, 0, 3, SOLVER>(e, p, step, nin, nout); break;
        default: launch_tile_k<T, 16, f32 ? 16 : 8, 1, R, 0, 4, SOLVER>(e, p, step, nin, nout); break;
    }
}

template <typename T, int SOLVER>
void go_fused_tile(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    if (e->geo.n[2] == 1) {
        if (e->R <= 1) go_tile2d<T, 1, SOLVER>(e, p, step, nin, nout);
        else go_tile2d<T, 2, SOLVER>(e, p, step, nin, nout);
        return;
    }
    if constexpr (sizeof(T) == 4) {
        switch (e->geo.nb) {
            case 1: launch_tile_k<T, 16, 8, 4, 1, 1, 1, SOLVER>(e, p, step, nin, nout); break;
            case 2: launch_tile_k<T, 16, 8, 4, 1, 1, 2, SOLVER>(e, p, step, nin, nout); break;
            default: launch_tile_k<T, 8, 8, 4, 1, 1, 3, SOLVER>(e, p, step, nin, nout); break;
        }
    } else {
        if (e->geo.nb == 1) launch_tile_k<T, 8, 8, 4, 1, 1, 1, SOLVER>(e, p, step, nin, nout);
        else launch_tile_k<T, 8, 8, 4, 1, 1, 2, SOLVER>(e, p, step, nin, nout);
    }
}

template <typename T>
void launch_tile(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    if (p->solver == SP_SOLVER_HEUN)
        go_fused_tile<T, sp::SOLVER_HEUN>(e, p, step, nin, nout);
    else if (p->solver == SP_SOLVER_SIB)
        go_fused_tile<T, sp::SOLVER_SIB>(e, p, step, nin, nout);
    else
        go_fused_tile<T, sp::SOLVER_DEPONDT>(e, p, step, nin, nout);
}

template <typename T, int TX, int TY, int TZ, int R, int RC, int NB>
void launch_gradient_tile_k(sp_engine* e, const void* n, void* g) {
    const dim3 grid((unsigned)((e->geo.n[0] + TX - 1) / TX), (unsigned)((e->geo.n[1] + TY - 1) / TY),
                    (unsigned)((e->geo.n[2] + TZ - 1) / TZ));
    constexpr int WN = TX + 2 * R, HN = TY + 2 * R, DN = TZ + 2 * RC;
    hipLaunchKernelGGL((sp::k_gradient_tile<T, TX, TY, TZ, R, RC, NB>), grid, dim3(NB * TX * TY * TZ), 0, e->stream,
                       make_stencilb<T>(e, WN, HN, WN * HN * DN, WN, HN, WN * HN * DN), make_siteb<T>(e, nullptr),
                       static_cast<const T*>(n), static_cast<T*>(g));
}

// The field of a lattice the fused tile path takes, on the same tiles.
template <typename T>
void launch_gradient_tile(sp_engine* e, const void* n, void* g) {
    constexpr bool f32 = sizeof(T) == 4;
    if (e->geo.n[2] == 1) {
        if (e->R <= 1) {
            switch (e->geo.nb) {
                case 2: launch_gradient_tile_k<T, f32 ? 32 : 16, 16, 1, 1, 0, 2>(e, n, g); break;
                case 3: launch_gradient_tile_k<T, 16, f32 ? 16 : 8, 1, 1, 0, 3>(e, n, g); break;
                default: launch_gradient_tile_k<T, 16, f32 ? 16 : 8, 1, 1, 0, 4>(e, n, g); break;
            }
        } else {
            switch (e->geo.nb) {
                case 2: launch_gradient_tile_k<T, f32 ? 32 : 16, 16, 1, 2, 0, 2>(e, n, g); break;
                case 3: launch_gradient_tile_k<T, 16, f32 ? 16 : 8, 1, 2, 0, 3>(e, n, g); break;
                default: launch_gradient_tile_k<T, 16, f32 ? 16 : 8, 1, 2, 0, 4>(e, n, g); break;
            }
        }
        return;
    }
    if constexpr (f32) {
        switch (e->geo.nb) {
            case 1: launch_gradient_tile_k<T, 16, 8, 4, 1, 1, 1>(e, n, g); break;
            case 2: launch_gradient_tile_k<T, 16, 8, 4, 1, 1, 2>(e, n, g); break;
            default: launch_gradient_tile_k<T, 8, 8, 4, 1, 1, 3>(e, n, g); break;
        }
    } else {
        if (e->geo.nb == 1) launch_gradient_tile_k<T, 8, 8, 4, 1, 1, 1>(e, n, g);
        else launch_gradient_tile_k<T, 8, 8, 4, 1, 1, 2>(e, n, g);
    }
}

// ------------------------------------------- compile-time-shape fused path
struct TileCfg {
    const char* name;
    int TX, TY, NT;
};
constexpr TileCfg kTileCfgs[] = {{"32x16x256", 32, 16, 256},  {"64x16x512", 64, 16, 512},
                                 {"32x16x512", 32, 16, 512},  {"32x32x1024", 32, 32, 1024},
                                 {"64x16x1024", 64, 16, 1024}, {"32x32x512", 32, 32, 512},
                                 {"64x16x256", 64, 16, 256}};
constexpr int kNumTileCfgs = 7;
constexpr int kNumTileCfgsF64 = 1;

template <int S>
bool match_shape(const sp_engine* e) {
    using SH = sp::ShapeTab<S>;
    if (e->n_shells != SH::NS || (int)e->all_bonds.size() != SH::NB) return false;
    for (int q = 0; q < SH::NB; ++q) {
        bool found = false;
        for (const HostBond& b : e->all_bonds)
            if (b.d[0] == SH::da[q] && b.d[1] == SH::db[q] && b.d[2] == 0 && b.shell == SH::sh[q]) found = true;
        if (!found) return false;
    }
    return true;
}

int detect_shape(const sp_engine* e) {
    if (match_shape<sp::SH_SQ1>(e)) return sp::SH_SQ1;
    if (match_shape<sp::SH_SQ2>(e)) return sp::SH_SQ2;
    if (match_shape<sp::SH_SQ3>(e)) return sp::SH_SQ3;
    if (match_shape<sp::SH_TRI1>(e)) return sp::SH_TRI1;
    if (match_shape<sp::SH_TRI2>(e)) return sp::SH_TRI2;
    if (match_shape<sp::SH_TRI3>(e)) return sp::SH_TRI3;
    return -1;
}

template <typename T, int S>
sp::ShapeCoef<T> shape_coef_for(const sp_engine* e) {
    using SH = sp::ShapeTab<S>;
    sp::ShapeCoef<T> C{};
    for (int s = 0; s < SH::NS; ++s) C.J[s] = (T)(s < e->ham.n_exch ? e->ham.J[s] : 0.0);
    for (int q = 0; q < SH::NB; ++q)
        for (const HostBond& b : e->all_bonds)
            if (b.d[0] == SH::da[q] && b.d[1] == SH::db[q] && b.shell == SH::sh[q]) {
                C.Dx[q] = (T)b.D[0];
                C.Dy[q] = (T)b.D[1];
            }
    return C;
}

// The step kernels' coefficients: those of shape_coef_for divided by
// mu mu_B (in double, then rounded), anisotropy likewise, and the external
// field in Tesla.
template <typename T, int S>
sp::StepCoef<T> step_coef_for(const sp_engine* e) {
    using SH = sp::ShapeTab<S>;
    const double inv = 1.0 / (e->ham.mu[0] * kMuB);
    const sp::ShapeCoef<double> D = shape_coef_for<double, S>(e);
    sp::StepCoef<T> C{};
    for (int s = 0; s < SH::NS; ++s) C.J[s] = (T)(D.J[s] * inv);
    for (int q = 0; q < SH::NB; ++q) {
        C.Dx[q] = (T)(D.Dx[q] * inv);
        C.Dy[q] = (T)(D.Dy[q] * inv);
    }
    C.K2 = (T)(2.0 * e->ham.K[0] * inv);
    for (int k = 0; k < 3; ++k) C.Bext[k] = (T)e->ham.B[k];
    return C;
}

template <typename T, int S, int NDMI, int TX, int TY, int NT, int SOLVER>
void go_shape(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    sp::TileMap M{};
    M.tiles_x = (e->geo.n[0] + TX - 1) / TX;
    M.tiles_y = (e->geo.n[1] + TY - 1) / TY;
    const int ntiles = M.tiles_x * M.tiles_y;
    M.xcd_bands = (ntiles >= 8 && ntiles % 8 == 0) ? 1 : 0;
    // FP32 Depondt on the 64 x 16 x 1024 tiles: a lattice periodic along both
    // axes (whose spins fit 32-bit byte offsets) takes the instance without
    // boundary tests
    if constexpr (sizeof(T) == 4 && SOLVER == sp::SOLVER_DEPONDT && TX == 64 && TY == 16 && NT == 1024) {
        const long long n_sites = (long long)e->geo.n[0] * e->geo.n[1];
        if (e->geo.per[0] && e->geo.per[1] && 3 * n_sites * (long long)sizeof(T) < (1ll << 32)) {
            hipLaunchKernelGGL((sp::k_fused2d_shape<T, S, NDMI, TX, TY, NT, SOLVER, true>), dim3((unsigned)ntiles),
                               dim3(NT), 0, e->stream, step_coef_for<T, S>(e), make_site2d<T>(e, p),
                               make_step_llg<T>(e, p, step), M, e->d_flag, static_cast<const T*>(nin),
                               static_cast<T*>(nout));
            return;
        }
    }
    hipLaunchKernelGGL((sp::k_fused2d_shape<T, S, NDMI, TX, TY, NT, SOLVER>), dim3((unsigned)ntiles), dim3(NT), 0, e->stream,
                       step_coef_for<T, S>(e), make_site2d<T>(e, p), make_step_llg<T>(e, p, step), M, e->d_flag,
                       static_cast<const T*>(nin), static_cast<T*>(nout));
}

template <typename T, int S, int TX, int TY, int NT, int SOLVER>
void go_ndmi(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    if (e->shape_ndmi)
        go_shape<T, S, sp::ShapeTab<S>::NB0, TX, TY, NT, SOLVER>(e, p, step, nin, nout);
    else
        go_shape<T, S, 0, TX, TY, NT, SOLVER>(e, p, step, nin, nout);
}

template <typename T, int TX, int TY, int NT, int SOLVER = sp::SOLVER_DEPONDT>
void go_tile(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    switch (e->shape) {
        case sp::SH_SQ1: go_ndmi<T, sp::SH_SQ1, TX, TY, NT, SOLVER>(e, p, step, nin, nout); break;
        case sp::SH_SQ2: go_ndmi<T, sp::SH_SQ2, TX, TY, NT, SOLVER>(e, p, step, nin, nout); break;
        case sp::SH_SQ3: go_ndmi<T, sp::SH_SQ3, TX, TY, NT, SOLVER>(e, p, step, nin, nout); break;
        case sp::SH_TRI1: go_ndmi<T, sp::SH_TRI1, TX, TY, NT, SOLVER>(e, p, step, nin, nout); break;
        case sp::SH_TRI2: go_ndmi<T, sp::SH_TRI2, TX, TY, NT, SOLVER>(e, p, step, nin, nout); break;
        default: go_ndmi<T, sp::SH_TRI3, TX, TY, NT, SOLVER>(e, p, step, nin, nout); break;
    }
}

// Heun and SIB run on one tile configuration per precision.
constexpr const char* kSolverTileF32 = "64x16x1024";
constexpr const char* kSolverTileF64 = "32x16x256";

template <typename T>
void launch_shape(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    if (p->solver == SP_SOLVER_HEUN) {
        if constexpr (sizeof(T) == 8)
            go_tile<T, 32, 16, 256, sp::SOLVER_HEUN>(e, p, step, nin, nout);
        else
            go_tile<T, 64, 16, 1024, sp::SOLVER_HEUN>(e, p, step, nin, nout);
        return;
    }
    if (p->solver == SP_SOLVER_SIB) {
        if constexpr (sizeof(T) == 8)
            go_tile<T, 32, 16, 256, sp::SOLVER_SIB>(e, p, step, nin, nout);
        else
            go_tile<T, 64, 16, 1024, sp::SOLVER_SIB>(e, p, step, nin, nout);
        return;
    }
    if constexpr (sizeof(T) == 8) {
        go_tile<T, 32, 16, 256>(e, p, step, nin, nout);
    } else {
        switch (e->tile_cfg) {
            case 1: go_tile<T, 64, 16, 512>(e, p, step, nin, nout); break;
            case 2: go_tile<T, 32, 16, 512>(e, p, step, nin, nout); break;
            case 3: go_tile<T, 32, 32, 1024>(e, p, step, nin, nout); break;
            case 4: go_tile<T, 64, 16, 1024>(e, p, step, nin, nout); break;
            case 5: go_tile<T, 32, 32, 512>(e, p, step, nin, nout); break;
            case 6: go_tile<T, 64, 16, 256>(e, p, step, nin, nout); break;
            default: go_tile<T, 32, 16, 256>(e, p, step, nin, nout); break;
        }
    }
}

// ------------------------------------------------ persistent 2D path
// Tiles of the persistent kernel (one thread per site); the matching
// one-step configuration of kTileCfgs serves single steps and the other
// solvers on this path.
struct PersistCfg {
    const char* name;
    int TX, TY;
    int tile_cfg;   // index of the same tile in kTileCfgs
    bool f64;       // offered in FP64
};
constexpr PersistCfg kPersistCfgs[] = {{"64x16", 64, 16, 4, false}, {"32x32", 32, 32, 3, false},
                                       {"32x16", 32, 16, 2, true}};
constexpr int kNumPersistCfgs = 3;
constexpr int kPersistSpinLimit = 1 << 21;   // polls per wait (~1 s) before a workgroup gives up
constexpr int kPersistMaxChunk = 1 << 16;    // steps per launch

template <typename T, int S, int NDMI, int TX, int TY>
int go_persist(sp_engine* e, const sp_llg_params* p, int n_steps, bool check_only) {
    const void* fn = reinterpret_cast<const void*>(&sp::k_persist2d<T, S, NDMI, TX, TY>);
    sp::PersistMap M{};
    M.tiles_x = e->geo.n[0] / TX;
    M.tiles_y = e->geo.n[1] / TY;
    const int ntiles = M.tiles_x * M.tiles_y;
    int per_cu = 0, n_cu = 0;
    HIPCHK(e, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, TX * TY, 0));
    HIPCHK(e, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, e->device));
    if ((long long)per_cu * n_cu < ntiles)
        return fail(e, SP_E_UNSUPPORTED, "persist2d needs every tile resident at once: " + std::to_string(ntiles) +
                                             " tiles, " + std::to_string((long long)per_cu * n_cu) + " slots");
    if (check_only) return SP_OK;
    if (ntiles > e->pflag_tiles || e->pgen > (1u << 30)) {
        int rc;
        if (ntiles > e->pflag_tiles) {
            if ((rc = dalloc(e, e->d_pflags, (size_t)ntiles * sp::kFlagStride * sizeof(uint32_t)))) return rc;
            e->pflag_tiles = ntiles;
        }
        HIPCHK(e, hipMemsetAsync(e->d_pflags, 0, (size_t)e->pflag_tiles * sp::kFlagStride * sizeof(uint32_t),
                                 e->stream));
        e->pgen = 0;
    }
    M.xcd_bands = (ntiles >= 8 && ntiles % 8 == 0) ? 1 : 0;
    M.n_steps = n_steps;
    M.gen = e->pgen;
    // SP_PERSIST_SPIN_LIMIT lowers the bound (tests of the time-out path)
    M.spin_limit = kPersistSpinLimit;
    if (const char* lim = std::getenv("SP_PERSIST_SPIN_LIMIT")) M.spin_limit = std::max(0, std::atoi(lim));
    sp::StepCoef<T> C = step_coef_for<T, S>(e);
    sp::Site2D<T> Q = make_site2d<T>(e, p);
    sp::LLGArgs<T> A = make_llg<T>(p, e->step, p->replica);
    const int* abort_flag = e->d_flag;
    T* b0 = static_cast<T*>(e->d_n);
    T* b1 = static_cast<T*>(e->d_n2);
    uint32_t* flags = e->d_pflags;
    int* status = e->d_pstatus;
    void* args[] = {&C, &Q, &A, &M, &abort_flag, &b0, &b1, &flags, &status};
    HIPCHK(e, hipLaunchCooperativeKernel(fn, dim3((unsigned)ntiles), dim3(TX * TY), args, 0, e->stream));
    e->pgen += (uint32_t)n_steps;
    if (n_steps & 1) std::swap(e->d_n, e->d_n2);
    e->step += (uint64_t)n_steps;
    return SP_OK;
}

template <typename T, int TX, int TY>
int go_persist_shape(sp_engine* e, const sp_llg_params* p, int n_steps, bool check_only) {
#define SP_PERSIST_CASE(SH)                                                                      \
    case SH:                                                                                     \
        return e->shape_ndmi ? go_persist<T, SH, sp::ShapeTab<SH>::NB0, TX, TY>(e, p, n_steps, check_only) \
                             : go_persist<T, SH, 0, TX, TY>(e, p, n_steps, check_only);
    switch (e->shape) {
        SP_PERSIST_CASE(sp::SH_SQ1)
        SP_PERSIST_CASE(sp::SH_SQ2)
        SP_PERSIST_CASE(sp::SH_SQ3)
        SP_PERSIST_CASE(sp::SH_TRI1)
        SP_PERSIST_CASE(sp::SH_TRI2)
        SP_PERSIST_CASE(sp::SH_TRI3)
        default: return fail(e, SP_E_UNSUPPORTED, "persist2d needs a compile-time stencil");
    }
#undef SP_PERSIST_CASE
}

// n_steps Depondt steps of the whole lattice in one launch (check_only:
// report whether the lattice and the tile fit the path, launch nothing).
template <typename T>
int launch_persist(sp_engine* e, const sp_llg_params* p, int n_steps, bool check_only = false) {
    const PersistCfg& c = kPersistCfgs[e->persist_cfg];
    if (e->shape < 0) return fail(e, SP_E_UNSUPPORTED, "persist2d needs a bond table matching a compile-time stencil");
    if (e->geo.n[0] % c.TX || e->geo.n[1] % c.TY)
        return fail(e, SP_E_UNSUPPORTED, std::string("persist2d/") + c.name + " needs lattice sides divisible by the tile");
    if (c.TX < 2 * e->R || c.TY < 2 * e->R) return fail(e, SP_E_UNSUPPORTED, "persist2d tile narrower than the halo");
    switch (e->persist_cfg) {
        case 0: if constexpr (sizeof(T) == 4) return go_persist_shape<T, 64, 16>(e, p, n_steps, check_only); break;
        case 1: if constexpr (sizeof(T) == 4) return go_persist_shape<T, 32, 32>(e, p, n_steps, check_only); break;
        default: return go_persist_shape<T, 32, 16>(e, p, n_steps, check_only);
    }
    return fail(e, SP_E_UNSUPPORTED, "persist2d tile not offered in this precision");
}

// ------------------------------------------------ 3D streamed fused path
// `blocks`: workgroups to aim for (the plane chunk length follows); tiles
// whose LDS rings leave room for several workgroups per CU aim higher.
struct Tile3Cfg {
    const char* name;
    int TX, TY, blocks;
};
constexpr Tile3Cfg kTile3Cfgs[] = {{"32x16", 32, 16, 256}, {"16x16", 16, 16, 768}, {"32x8", 32, 8, 768},
                                   {"16x16z", 16, 16, 256}, {"32x16b", 32, 16, 512}, {"32x32", 32, 32, 256}};
constexpr int kNumTile3Cfgs = 6;      // FP64 takes the 16x16 tiles only (LDS)

template <int S>
bool match_shape3(const sp_engine* e) {
    using SH = sp::ShapeTab3<S>;
    if (e->n_shells != SH::NS || (int)e->all_bonds.size() != SH::NB) return false;
    for (int q = 0; q < SH::NB; ++q) {
        bool found = false;
        for (const HostBond& b : e->all_bonds)
            if (b.d[0] == SH::da[q] && b.d[1] == SH::db[q] && b.d[2] == SH::dc[q] && b.shell == SH::sh[q]) found = true;
        if (!found) return false;
    }
    return true;
}

int detect_shape3(const sp_engine* e) {
    if (match_shape3<sp::SH3_SC1>(e)) return sp::SH3_SC1;
    if (match_shape3<sp::SH3_SC2>(e)) return sp::SH3_SC2;
    if (match_shape3<sp::SH3_SC3>(e)) return sp::SH3_SC3;
    return -1;
}

// Whether the six nearest-neighbour bonds carry the bulk DMI form
// D_b = D0 (da, db, dc) (simple cubic, unit bond vectors) with one D0;
// *D0 receives it.
bool bulk_dmi3(const std::vector<HostBond>& bonds, double* D0) {
    double d0 = 0.0;
    bool have = false;
    int found = 0;
    for (const HostBond& b : bonds) {
        if (b.shell != 0) continue;
        const int L1 = std::abs(b.d[0]) + std::abs(b.d[1]) + std::abs(b.d[2]);
        if (L1 != 1) return false;
        const double c = b.d[0] * b.D[0] + b.d[1] * b.D[1] + b.d[2] * b.D[2];
        if (!have) {
            d0 = c;
            have = true;
        }
        for (int k = 0; k < 3; ++k)
            if (std::fabs(b.D[k] - d0 * b.d[k]) > 1e-14 * std::fabs(d0)) return false;
        ++found;
    }
    if (found != 6 || d0 == 0.0) return false;
    if (D0) *D0 = d0;
    return true;
}

template <typename T, int S>
sp::ShapeCoef3<T> shape_coef3_for(const sp_engine* e) {
    using SH = sp::ShapeTab3<S>;
    sp::ShapeCoef3<T> C{};
    for (int s = 0; s < SH::NS; ++s) C.J[s] = (T)(s < e->ham.n_exch ? e->ham.J[s] : 0.0);
    for (int q = 0; q < SH::NB0; ++q)
        for (const HostBond& b : e->all_bonds)
            if (b.d[0] == SH::da[q] && b.d[1] == SH::db[q] && b.d[2] == SH::dc[q] && b.shell == 0) {
                C.Dx[q] = (T)b.D[0];
                C.Dy[q] = (T)b.D[1];
                C.Dz[q] = (T)b.D[2];
            }
    double d0 = 0.0;
    if (bulk_dmi3(e->all_bonds, &d0)) C.D0 = (T)d0;
    return C;
}

// The step kernel's coefficients: those of shape_coef3_for divided by
// mu mu_B (in double, then rounded), and the external field in Tesla.
template <typename T, int S>
sp::StepCoef3<T> step_coef3_for(const sp_engine* e) {
    using SH = sp::ShapeTab3<S>;
    const double inv = 1.0 / (e->ham.mu[0] * kMuB);
    const sp::ShapeCoef3<double> D = shape_coef3_for<double, S>(e);
    sp::StepCoef3<T> C{};
    for (int s = 0; s < SH::NS; ++s) C.J[s] = (T)(D.J[s] * inv);
    for (int q = 0; q < SH::NB0; ++q) {
        C.Dx[q] = (T)(D.Dx[q] * inv);
        C.Dy[q] = (T)(D.Dy[q] * inv);
        C.Dz[q] = (T)(D.Dz[q] * inv);
    }
    C.D0 = (T)(D.D0 * inv);
    C.K2 = (T)(2.0 * e->ham.K[0] * inv);
    for (int k = 0; k < 3; ++k) C.Bext[k] = (T)e->ham.B[k];
    return C;
}

template <typename T, int S, int DK, int TX, int TY, int SOLVER>
void go_shape3(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    const int target = kTile3Cfgs[e->tile3_cfg].blocks;
    sp::Site3D Z{};
    Z.nc = e->geo.n[2];
    Z.per_c = e->geo.per[2];
    Z.tiles_x = (e->geo.n[0] + TX - 1) / TX;
    Z.tiles_y = (e->geo.n[1] + TY - 1) / TY;
    const int txy = Z.tiles_x * Z.tiles_y;
    const int chunks = std::max(1, std::min(Z.nc, (target + txy - 1) / txy));
    Z.zc = (Z.nc + chunks - 1) / chunks;
    const int nchunks = (Z.nc + Z.zc - 1) / Z.zc;
    Z.xcd_bands = ((txy * nchunks) % 8 == 0) ? 1 : 0;
    const dim3 grid((unsigned)(txy * nchunks)), block(TX * TY);
    // Depondt steps without anisotropy take the instance that leaves the term
    // out; on the 32 x 32 columns a lattice periodic along every axis (whose
    // spins fit 32-bit byte offsets) takes the instance without boundary tests
    if constexpr (SOLVER == sp::SOLVER_DEPONDT && TX * TY == 1024) {
        const long long n_sites = (long long)e->geo.n[0] * e->geo.n[1] * e->geo.n[2];
        if (e->geo.per[0] && e->geo.per[1] && e->geo.per[2] && 3 * n_sites * (long long)sizeof(T) < (1ll << 32)) {
            if (e->ham.K[0] == 0.0)
                hipLaunchKernelGGL((sp::k_fused3d_shape<T, S, DK, TX, TY, SOLVER, false, true>), grid, block, 0,
                                   e->stream, step_coef3_for<T, S>(e), make_site2d<T>(e, p), Z,
                                   make_step_llg<T>(e, p, step), e->d_flag, static_cast<const T*>(nin),
                                   static_cast<T*>(nout));
            else
                hipLaunchKernelGGL((sp::k_fused3d_shape<T, S, DK, TX, TY, SOLVER, true, true>), grid, block, 0,
                                   e->stream, step_coef3_for<T, S>(e), make_site2d<T>(e, p), Z,
                                   make_step_llg<T>(e, p, step), e->d_flag, static_cast<const T*>(nin),
                                   static_cast<T*>(nout));
            return;
        }
    }
    if constexpr (SOLVER == sp::SOLVER_DEPONDT) {
        if (e->ham.K[0] == 0.0) {
            hipLaunchKernelGGL((sp::k_fused3d_shape<T, S, DK, TX, TY, SOLVER, false>), grid, block, 0, e->stream,
                               step_coef3_for<T, S>(e), make_site2d<T>(e, p), Z, make_step_llg<T>(e, p, step),
                               e->d_flag, static_cast<const T*>(nin), static_cast<T*>(nout));
            return;
        }
    }
    hipLaunchKernelGGL((sp::k_fused3d_shape<T, S, DK, TX, TY, SOLVER, true>), grid, block, 0, e->stream,
                       step_coef3_for<T, S>(e), make_site2d<T>(e, p), Z, make_step_llg<T>(e, p, step), e->d_flag,
                       static_cast<const T*>(nin), static_cast<T*>(nout));
}

template <typename T, int S, int TX, int TY, int SOLVER>
void go_dk3(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    if (e->shape3_dk == sp::DK_BULK)
        go_shape3<T, S, sp::DK_BULK, TX, TY, SOLVER>(e, p, step, nin, nout);
    else if (e->shape3_dk == sp::DK_GENERAL)
        go_shape3<T, S, sp::DK_GENERAL, TX, TY, SOLVER>(e, p, step, nin, nout);
    else
        go_shape3<T, S, sp::DK_NONE, TX, TY, SOLVER>(e, p, step, nin, nout);
}

template <typename T, int TX, int TY, int SOLVER>
void go_tile3(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    switch (e->shape3) {
        case sp::SH3_SC1: go_dk3<T, sp::SH3_SC1, TX, TY, SOLVER>(e, p, step, nin, nout); break;
        case sp::SH3_SC2: go_dk3<T, sp::SH3_SC2, TX, TY, SOLVER>(e, p, step, nin, nout); break;
        default: go_dk3<T, sp::SH3_SC3, TX, TY, SOLVER>(e, p, step, nin, nout); break;
    }
}

template <typename T, int SOLVER>
void go_cfg3(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    if constexpr (sizeof(T) == 8) {
        go_tile3<T, 16, 16, SOLVER>(e, p, step, nin, nout);
    } else {
        if (e->tile3_cfg == 1 || e->tile3_cfg == 3)
            go_tile3<T, 16, 16, SOLVER>(e, p, step, nin, nout);
        else if (e->tile3_cfg == 2)
            go_tile3<T, 32, 8, SOLVER>(e, p, step, nin, nout);
        else if (e->tile3_cfg == 5)
            go_tile3<T, 32, 32, SOLVER>(e, p, step, nin, nout);
        // configurations 0 and 4 share the 32x16 kernel (different chunking)
        else
            go_tile3<T, 32, 16, SOLVER>(e, p, step, nin, nout);
    }
}

template <typename T>
void launch_shape3(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    if (p->solver == SP_SOLVER_HEUN)
        go_cfg3<T, sp::SOLVER_HEUN>(e, p, step, nin, nout);
    else if (p->solver == SP_SOLVER_SIB)
        go_cfg3<T, sp::SOLVER_SIB>(e, p, step, nin, nout);
    else
        go_cfg3<T, sp::SOLVER_DEPONDT>(e, p, step, nin, nout);
}

template <typename T>
int launch_step(sp_engine* e, const sp_llg_params* p, uint64_t step, const void* nin, void* nout) {
    if (std::strcmp(e->path, "shape2d") == 0 || std::strcmp(e->path, "persist2d") == 0) {
        launch_shape<T>(e, p, step, nin, nout);
        HIPCHK(e, hipGetLastError());
        return SP_OK;
    }
    if (std::strcmp(e->path, "shape3d") == 0) {
        launch_shape3<T>(e, p, step, nin, nout);
        HIPCHK(e, hipGetLastError());
        return SP_OK;
    }
    if (std::strcmp(e->path, "fusedtile") == 0) {
        launch_tile<T>(e, p, step, nin, nout);
        HIPCHK(e, hipGetLastError());
        return SP_OK;
    }
    if (std::strcmp(e->path, "fused2d") == 0 && p->solver == SP_SOLVER_DEPONDT) {
        if (e->R <= 1)
            launch_fused2d<T, 32, 16, 1>(e, p, step, nin, nout);
        else
            launch_fused2d<T, 32, 16, 2>(e, p, step, nin, nout);
        HIPCHK(e, hipGetLastError());
        return SP_OK;
    }
    const sp::Lattice L = make_lattice(e);
    const sp::BondCoef<T> C = make_coef<T>(e);
    const sp::Phys<T> P = make_phys<T>(e, p);
    const sp::LLGArgs<T> A = make_step_llg<T>(e, p, step);
    const void* gdd = nullptr;
    const void* gddp = nullptr;
    if (e->ham.ddi) {
        int rc = launch_dipole<T>(e, nin, e->d_gdd);
        if (rc) return rc;
        gdd = e->d_gdd;
    }
    const dim3 grid(blocks_for(e->N)), block(256);
    if (p->solver == SP_SOLVER_HEUN)
        hipLaunchKernelGGL((sp::k_predict<T, sp::SOLVER_HEUN>), grid, block, 0, e->stream, L, C, P, A, e->d_flag,
                           static_cast<const T*>(nin), static_cast<const T*>(gdd), static_cast<T*>(e->d_np),
                           static_cast<T*>(e->d_A));
    else if (p->solver == SP_SOLVER_SIB)
        hipLaunchKernelGGL((sp::k_predict<T, sp::SOLVER_SIB>), grid, block, 0, e->stream, L, C, P, A, e->d_flag,
                           static_cast<const T*>(nin), static_cast<const T*>(gdd), static_cast<T*>(e->d_np),
                           static_cast<T*>(e->d_A));
    else
        hipLaunchKernelGGL((sp::k_predict<T, sp::SOLVER_DEPONDT>), grid, block, 0, e->stream, L, C, P, A, e->d_flag,
                           static_cast<const T*>(nin), static_cast<const T*>(gdd), static_cast<T*>(e->d_np),
                           static_cast<T*>(e->d_A));
    if (e->ham.ddi) {
        // the corrector's dipole field is evaluated on what the predictor
        // stored: n^p (Depondt, Heun) or the midpoint (SIB)
        int rc = launch_dipole<T>(e, e->d_np, e->d_gddp);
        if (rc) return rc;
        gddp = e->d_gddp;
    }
    if (p->solver == SP_SOLVER_HEUN)
        hipLaunchKernelGGL((sp::k_correct<T, sp::SOLVER_HEUN>), grid, block, 0, e->stream, L, C, P, A, e->d_flag,
                           static_cast<const T*>(nin), static_cast<const T*>(e->d_np), static_cast<const T*>(gddp),
                           static_cast<const T*>(e->d_A), static_cast<T*>(nout));
    else if (p->solver == SP_SOLVER_SIB)
        hipLaunchKernelGGL((sp::k_correct<T, sp::SOLVER_SIB>), grid, block, 0, e->stream, L, C, P, A, e->d_flag,
                           static_cast<const T*>(nin), static_cast<const T*>(e->d_np), static_cast<const T*>(gddp),
                           static_cast<const T*>(e->d_A), static_cast<T*>(nout));
    else
        hipLaunchKernelGGL((sp::k_correct<T, sp::SOLVER_DEPONDT>), grid, block, 0, e->stream, L, C, P, A, e->d_flag,
                           static_cast<const T*>(nin), static_cast<const T*>(e->d_np), static_cast<const T*>(gddp),
                           static_cast<const T*>(e->d_A), static_cast<T*>(nout));
    HIPCHK(e, hipGetLastError());
    return SP_OK;
}

int check_ready(sp_engine* e, bool need_spins) {
    if (!e) return SP_E_ARG;
    if (!e->has_geo) return fail(e, SP_E_ORDER, "sp_set_geometry has not been called");
    if (!e->has_ham) return fail(e, SP_E_ORDER, "sp_set_hamiltonian has not been called");
    if (need_spins && !e->has_spins) return fail(e, SP_E_ORDER, "sp_set_spins has not been called");
    return SP_OK;
}

int check_llg(sp_engine* e, const sp_llg_params* p) {
    if (!p) return fail(e, SP_E_ARG, "llg params are NULL");
    if (!(p->alpha >= 0.0) || !std::isfinite(p->alpha)) return fail(e, SP_E_ARG, "alpha must be finite and >= 0");
    if (!(p->dt_ps > 0.0) || !std::isfinite(p->dt_ps)) return fail(e, SP_E_ARG, "dt must be finite and > 0");
    if (!(p->T_K >= 0.0) || !std::isfinite(p->T_K)) return fail(e, SP_E_ARG, "T must be finite and >= 0");
    if (p->solver != SP_SOLVER_DEPONDT && p->solver != SP_SOLVER_HEUN && p->solver != SP_SOLVER_SIB)
        return fail(e, SP_E_ARG, "solver must be SP_SOLVER_DEPONDT, SP_SOLVER_HEUN or SP_SOLVER_SIB");
    return SP_OK;
}

template <typename T>
int copy_in_soa(sp_engine* e, void* dst, const double* src, int64_t n3) {
    if constexpr (sizeof(T) == 8) {
        HIPCHK(e, hipMemcpyAsync(dst, src, n3 * sizeof(double), hipMemcpyHostToDevice, e->stream));
    } else {
        std::vector<float> tmp((size_t)n3);
        for (int64_t k = 0; k < n3; ++k) tmp[k] = (float)src[k];
        HIPCHK(e, hipMemcpyAsync(dst, tmp.data(), n3 * sizeof(float), hipMemcpyHostToDevice, e->stream));
        HIPCHK(e, hipStreamSynchronize(e->stream));
    }
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return SP_OK;
}

template <typename T>
int copy_out_soa(sp_engine* e, double* dst, const void* src, int64_t n3) {
    if constexpr (sizeof(T) == 8) {
        HIPCHK(e, hipMemcpyAsync(dst, src, n3 * sizeof(double), hipMemcpyDeviceToHost, e->stream));
        HIPCHK(e, hipStreamSynchronize(e->stream));
    } else {
        std::vector<float> tmp((size_t)n3);
        HIPCHK(e, hipMemcpyAsync(tmp.data(), src, n3 * sizeof(float), hipMemcpyDeviceToHost, e->stream));
        HIPCHK(e, hipStreamSynchronize(e->stream));
        for (int64_t k = 0; k < n3; ++k) dst[k] = (double)tmp[k];
    }
    return SP_OK;
}

template <typename T>
int upload_ham(sp_engine* e) {
    const size_t nbond = e->bonds.size();
    std::vector<int4> bd(std::max<size_t>(nbond, 1));
    std::vector<T> J(std::max<size_t>(nbond, 1)), D(3 * std::max<size_t>(nbond, 1));
    for (size_t q = 0; q < nbond; ++q) {
        const HostBond& b = e->bonds[q];
        bd[q] = make_int4(b.bj, b.d[0], b.d[1], b.d[2]);
        J[q] = (T)b.J;
        for (int k = 0; k < 3; ++k) D[3 * q + k] = (T)b.D[k];
    }
    int rc;
    if ((rc = dalloc(e, e->d_bond, bd.size() * sizeof(int4)))) return rc;
    if ((rc = dalloc(e, e->d_bstart, e->bstart.size() * sizeof(int)))) return rc;
    if ((rc = dalloc(e, e->d_J, J.size() * sizeof(T)))) return rc;
    if ((rc = dalloc(e, e->d_D, D.size() * sizeof(T)))) return rc;
    HIPCHK(e, hipMemcpy(e->d_bond, bd.data(), bd.size() * sizeof(int4), hipMemcpyHostToDevice));
    HIPCHK(e, hipMemcpy(e->d_bstart, e->bstart.data(), e->bstart.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(e, hipMemcpy(e->d_J, J.data(), J.size() * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(e, hipMemcpy(e->d_D, D.data(), D.size() * sizeof(T), hipMemcpyHostToDevice));
    if constexpr (sizeof(T) == 4) {
        std::vector<double> J64(J.size()), D64(D.size());
        for (size_t q = 0; q < nbond; ++q) {
            J64[q] = e->bonds[q].J;
            for (int k = 0; k < 3; ++k) D64[3 * q + k] = e->bonds[q].D[k];
        }
        if ((rc = dalloc(e, e->d_J64, J64.size() * sizeof(double)))) return rc;
        if ((rc = dalloc(e, e->d_D64, D64.size() * sizeof(double)))) return rc;
        HIPCHK(e, hipMemcpy(e->d_J64, J64.data(), J64.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(e, hipMemcpy(e->d_D64, D64.data(), D64.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if (e->ham.ddi) {
        // site positions in Angstrom
        std::vector<T> pos(3 * (size_t)e->N);
        const HostGeo& g = e->geo;
        for (int i = 0; i < e->N; ++i) {
            const int a = i % g.n[0];
            const int b = (i / g.n[0]) % g.n[1];
            const int c = (i / (g.n[0] * g.n[1])) % g.n[2];
            const int beta = i / (g.n[0] * g.n[1] * g.n[2]);
            for (int k = 0; k < 3; ++k)
                pos[(size_t)k * e->N + i] =
                    (T)((a * g.bravais[k] + b * g.bravais[3 + k] + c * g.bravais[6 + k] + g.basis[3 * beta + k]) * g.a);
        }
        if ((rc = dalloc(e, e->d_pos, pos.size() * sizeof(T)))) return rc;
        HIPCHK(e, hipMemcpy(e->d_pos, pos.data(), pos.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    return SP_OK;
}

// Stencil gradient of a one-atom 2D lattice with a compile-time stencil:
// 64 x 16 tiles with one site per thread, or, for FP32 lattices of at least
// 512 such 64 x 64 tiles, 64 x 64 tiles with four sites per thread (more
// loads in flight per CU, less halo).
template <typename T, int S, int TX, int TY, int NT>
void go_gradient_tile(sp_engine* e, const void* n, void* g) {
    sp::TileMap M{};
    M.tiles_x = (e->geo.n[0] + TX - 1) / TX;
    M.tiles_y = (e->geo.n[1] + TY - 1) / TY;
    const int ntiles = M.tiles_x * M.tiles_y;
    M.xcd_bands = (ntiles >= 8 && ntiles % 8 == 0) ? 1 : 0;
    const sp::ShapeCoef<T> C = shape_coef_for<T, S>(e);
    const sp::Site2D<T> Q = make_site2d<T>(e, nullptr);
    if (e->shape_ndmi)
        hipLaunchKernelGGL((sp::k_gradient_shape<T, S, sp::ShapeTab<S>::NB0, TX, TY, NT>), dim3((unsigned)ntiles),
                           dim3(NT), 0, e->stream, C, Q, M, static_cast<const T*>(n), static_cast<T*>(g));
    else
        hipLaunchKernelGGL((sp::k_gradient_shape<T, S, 0, TX, TY, NT>), dim3((unsigned)ntiles), dim3(NT), 0,
                           e->stream, C, Q, M, static_cast<const T*>(n), static_cast<T*>(g));
}

template <typename T, int S>
void go_gradient_shape(sp_engine* e, const void* n, void* g) {
    const long long big_tiles = (long long)((e->geo.n[0] + 63) / 64) * ((e->geo.n[1] + 63) / 64);
    if constexpr (sizeof(T) == 4) {
        if (big_tiles >= 512 && e->geo.n[0] % 64 == 0 && e->geo.n[1] % 64 == 0 &&
            reinterpret_cast<uintptr_t>(n) % 16 == 0 && reinterpret_cast<uintptr_t>(g) % 16 == 0) {
            // whole 64 x 64 tiles and 16-byte aligned arrays: 16-byte loads and stores
            sp::TileMap M{};
            M.tiles_x = e->geo.n[0] / 64;
            M.tiles_y = e->geo.n[1] / 64;
            const int ntiles = M.tiles_x * M.tiles_y;
            M.xcd_bands = ntiles % 8 == 0 ? 1 : 0;
            const sp::ShapeCoef<float> C = shape_coef_for<float, S>(e);
            const sp::Site2D<float> Q = make_site2d<float>(e, nullptr);
            if (e->shape_ndmi)
                hipLaunchKernelGGL((sp::k_gradient_shape_v4<S, sp::ShapeTab<S>::NB0>), dim3((unsigned)ntiles), dim3(1024),
                                   0, e->stream, C, Q, M, static_cast<const float*>(n), static_cast<float*>(g));
            else
                hipLaunchKernelGGL((sp::k_gradient_shape_v4<S, 0>), dim3((unsigned)ntiles), dim3(1024), 0, e->stream, C,
                                   Q, M, static_cast<const float*>(n), static_cast<float*>(g));
            return;
        }
        if (big_tiles >= 512) {
            go_gradient_tile<T, S, 64, 64, 1024>(e, n, g);
            return;
        }
    }
    go_gradient_tile<T, S, 64, 16, 1024>(e, n, g);
}

template <typename T>
int gradient_dev(sp_engine* e, const void* n, void* g) {
    if (e->shape >= 0) {   // no dipole, no on-site potentials on this path
        switch (e->shape) {
            case sp::SH_SQ1: go_gradient_shape<T, sp::SH_SQ1>(e, n, g); break;
            case sp::SH_SQ2: go_gradient_shape<T, sp::SH_SQ2>(e, n, g); break;
            case sp::SH_SQ3: go_gradient_shape<T, sp::SH_SQ3>(e, n, g); break;
            case sp::SH_TRI1: go_gradient_shape<T, sp::SH_TRI1>(e, n, g); break;
            case sp::SH_TRI2: go_gradient_shape<T, sp::SH_TRI2>(e, n, g); break;
            default: go_gradient_shape<T, sp::SH_TRI3>(e, n, g); break;
        }
        HIPCHK(e, hipGetLastError());
        return SP_OK;
    }
    if (e->tile_ok) {   // lattices with a basis: LDS tiles (no dipole, no on-site potentials)
        launch_gradient_tile<T>(e, n, g);
        HIPCHK(e, hipGetLastError());
        return SP_OK;
    }
    const void* gdd = nullptr;
    if (e->ham.ddi) {
        int rc = launch_dipole<T>(e, n, e->d_gdd);
        if (rc) return rc;
        gdd = e->d_gdd;
    }
    hipLaunchKernelGGL((sp::k_gradient<T>), dim3(blocks_for(e->N)), dim3(256), 0, e->stream, make_lattice(e),
                       make_coef<T>(e), make_phys<T>(e, nullptr), static_cast<const T*>(n),
                       static_cast<const T*>(gdd), static_cast<T*>(g));
    HIPCHK(e, hipGetLastError());
    return SP_OK;
}

template <typename T>
int normals_dev(sp_engine* e, uint64_t seed, uint64_t step, uint32_t replica, uint32_t site0, int64_t n,
                double* eta, uint32_t* raw) {
    void* d_eta = nullptr;
    uint32_t* d_raw = nullptr;
    int rc;
    if ((rc = dalloc(e, d_eta, 3 * (size_t)n * sizeof(T)))) return rc;
    if ((rc = dalloc(e, d_raw, 4 * (size_t)n * sizeof(uint32_t)))) { dfree(d_eta); return rc; }
    sp::ThermalKey k{(uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)step, (uint32_t)(step >> 32), replica};
    hipLaunchKernelGGL((sp::k_normals<T>), dim3(blocks_for(n)), dim3(256), 0, e->stream, k, site0, (int)n,
                       static_cast<T*>(d_eta), d_raw);
    rc = copy_out_soa<T>(e, eta, d_eta, 3 * n);
    if (rc == SP_OK && raw) {
        hipError_t s = hipMemcpy(raw, d_raw, 4 * (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (s != hipSuccess) rc = fail(e, SP_E_HIP, hipGetErrorString(s));
    }
    dfree(d_eta);
    void* r = d_raw;
    dfree(r);
    return rc;
}

// Graph replay of sp_run.  Steps are grouped into chunks of C steps (the
// observation interval, or kGraphChunk when nothing is observed); a chunk is
// captured once as a HIP graph (C step launches, the observation, and a
// one-thread kernel that advances the device step and files the observation)
// and replayed for every later chunk with the same parameters, buffers and
// step path.  The step kernels of a replayed chunk read the Philox step from
// the device counter, so the replays reproduce the direct launches bit for bit.
constexpr int64_t kGraphChunk = 32;
constexpr int64_t kGraphMaxChunk = 1024;
constexpr size_t kGraphCache = 8;

bool same_params(const sp_llg_params& a, const sp_llg_params& b) {
    return a.alpha == b.alpha && a.dt_ps == b.dt_ps && a.T_K == b.T_K && a.seed == b.seed &&
           a.replica == b.replica && a.solver == b.solver;
}

std::string path_key(const sp_engine* e) {
    return std::string(e->path) + "/" + std::to_string(e->tile_cfg) + "/" + std::to_string(e->tile3_cfg);
}

template <typename T>
int capture_chunk(sp_engine* e, const sp_llg_params* p, int C, bool observe, double tol, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    HIPCHK(e, hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
    void* a = e->d_n;
    void* b = e->d_n2;
    int rc = SP_OK;
    e->cap_step_dev = e->d_step;
    for (int k = 0; k < C && rc == SP_OK; ++k) {
        e->cap_step_off = (unsigned int)k;
        rc = launch_step<T>(e, p, e->step + (uint64_t)k, a, b);
        std::swap(a, b);
    }
    e->cap_step_dev = nullptr;
    e->cap_step_off = 0;
    if (rc == SP_OK && observe) rc = launch_observe<T>(e, a, e->d_obs_stage, 0, true, e->d_step, C, tol);
    if (rc == SP_OK)
        hipLaunchKernelGGL(sp::k_run_chunk_end, dim3(1), dim3(64), 0, e->stream, e->d_step, e->d_obs_index,
                           observe ? (const double*)e->d_obs_stage : nullptr, e->d_obs, (long long)e->obs_cap, C);
    const hipError_t st = hipStreamEndCapture(e->stream, &g);
    if (rc != SP_OK || st != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return rc != SP_OK ? rc : fail(e, SP_E_HIP, std::string("step graph capture: ") + hipGetErrorString(st));
    }
    hipGraphExec_t x = nullptr;
    const hipError_t si = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (si != hipSuccess) return fail(e, SP_E_HIP, std::string("step graph instantiate: ") + hipGetErrorString(si));
    *out = x;
    return SP_OK;
}

template <typename T>
int chunk_graph(sp_engine* e, const sp_llg_params* p, int C, bool observe, double tol, hipGraphExec_t* out) {
    const std::string pk = path_key(e);
    for (const RunGraph& g : e->graphs)
        if (same_params(g.p, *p) && g.steps == C && g.observe == observe && g.tol == tol && g.n_first == e->d_n &&
            g.n_other == e->d_n2 && g.obs == e->d_obs && g.obs_cap == e->obs_cap && g.path == pk) {
            *out = g.exec;
            return SP_OK;
        }
    hipGraphExec_t x = nullptr;
    int rc = capture_chunk<T>(e, p, C, observe, tol, &x);
    if (rc) return rc;
    if (e->graphs.size() >= kGraphCache) {
        (void)hipGraphExecDestroy(e->graphs.front().exec);
        e->graphs.erase(e->graphs.begin());
    }
    e->graphs.push_back(RunGraph{*p, C, observe, tol, e->d_n, e->d_n2, e->d_obs, (long long)e->obs_cap, pk, x});
    *out = x;
    return SP_OK;
}

// Runs n_steps steps (or fewer: a non-finite torque aborts the run, and with
// tol > 0 an observation whose maximum torque is below tol stops it).  The
// decision is taken on the device; the host reads it once at the end.
template <typename T>
int run_impl(sp_engine* e, const sp_llg_params* p, int64_t n_steps, int64_t observe_every, double tol,
             sp_observation* obs, int64_t* steps_done) {
    const int64_t n_obs = observe_every > 0 ? n_steps / observe_every : 0;
    int rc;
    if (n_obs > e->obs_cap) {
        if ((rc = dalloc(e, e->d_obs, (size_t)n_obs * sp::OBS_NVALS * sizeof(double)))) return rc;
        e->obs_cap = n_obs;
    }
    sp::k_set_run_ctl<<<1, 64, 0, e->stream>>>(e->d_flag, e->d_abort_step, e->d_step, e->d_obs_index,
                                               (unsigned long long)e->step, 0LL);
    HIPCHK(e, hipGetLastError());
    const uint64_t step0 = e->step;
    int64_t k = 0;
    const bool persist = std::strcmp(e->path, "persist2d") == 0 && p->solver == SP_SOLVER_DEPONDT;
    if (persist) {
        HIPCHK(e, hipMemsetAsync(e->d_pstatus, 0, sizeof(int), e->stream));
        // one launch per observation interval (or per kPersistMaxChunk steps)
        for (int64_t t = 0; t < n_steps;) {
            int64_t chunk = observe_every > 0 ? observe_every - t % observe_every : n_steps - t;
            chunk = std::min<int64_t>(std::min<int64_t>(chunk, n_steps - t), kPersistMaxChunk);
            if ((rc = launch_persist<T>(e, p, (int)chunk))) return rc;
            t += chunk;
            if (observe_every > 0 && t % observe_every == 0) {
                rc = launch_observe<T>(e, e->d_n, e->d_obs + k * sp::OBS_NVALS, (long long)e->step, true, nullptr,
                                       0, tol);
                if (rc) return rc;
                ++k;
            }
        }
    }
    int64_t t = 0;
    const int64_t C = observe_every > 0 ? observe_every : kGraphChunk;
    if (!persist && e->graphs_on && !e->ham.ddi && C <= kGraphMaxChunk && n_steps >= C) {
        for (const int64_t chunks = n_steps / C; t < chunks * C; t += C) {
            hipGraphExec_t x = nullptr;
            if ((rc = chunk_graph<T>(e, p, (int)C, observe_every > 0, tol, &x))) return rc;
            HIPCHK(e, hipGraphLaunch(x, e->stream));
            if (C % 2) std::swap(e->d_n, e->d_n2);
            e->step += (uint64_t)C;
            if (observe_every > 0) ++k;
        }
    }
    for (; !persist && t < n_steps; ++t) {
        rc = launch_step<T>(e, p, e->step, e->d_n, e->d_n2);
        if (rc) return rc;
        std::swap(e->d_n, e->d_n2);
        ++e->step;
        if (observe_every > 0 && (t + 1) % observe_every == 0) {
            rc = launch_observe<T>(e, e->d_n, e->d_obs + k * sp::OBS_NVALS, (long long)e->step, true, nullptr, 0,
                                   tol);
            if (rc) return rc;
            ++k;
        }
    }
    int flag = 0;
    long long astep = 0;
    HIPCHK(e, hipMemcpyAsync(&flag, e->d_flag, sizeof(int), hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipMemcpyAsync(&astep, e->d_abort_step, sizeof(long long), hipMemcpyDeviceToHost, e->stream));
    std::vector<double> h((size_t)n_obs * sp::OBS_NVALS);
    if (n_obs > 0 && obs)
        HIPCHK(e, hipMemcpyAsync(h.data(), e->d_obs, h.size() * sizeof(double), hipMemcpyDeviceToHost, e->stream));
    HIPCHK(e, hipStreamSynchronize(e->stream));
    if (persist) {
        int pst = 0;
        HIPCHK(e, hipMemcpy(&pst, e->d_pstatus, sizeof(int), hipMemcpyDeviceToHost));
        if (pst) {
            // flags may have stopped anywhere: start the next launch from zero
            e->pgen = (1u << 30) + 1;
            return fail(e, SP_E_HIP, "persist2d: a tile timed out waiting for its neighbours; spins are invalid");
        }
    }
    int64_t done = n_steps;
    if (flag == sp::RUN_CONVERGED) {
        // the steps after the converged observation were skipped: the state
        // is the one observed, and the buffers swapped once per skipped step
        done = (int64_t)(astep - (long long)step0);
        if ((n_steps - done) % 2) std::swap(e->d_n, e->d_n2);
        e->step = step0 + (uint64_t)done;
    }
    if (steps_done) *steps_done = done;
    if (n_obs > 0 && obs) {
        const int64_t n_kept = observe_every > 0 ? std::min<int64_t>(n_obs, done / observe_every) : 0;
        for (int64_t q = 0; q < n_kept; ++q)
            obs_from(&h[(size_t)q * sp::OBS_NVALS], (int64_t)step0 + (q + 1) * observe_every, e->N, &obs[q]);
    }
    if (flag == sp::RUN_NONFINITE)
        return fail(e, SP_E_NONFINITE, "non-finite torque observed after step " + std::to_string(astep) +
                                           "; later steps were skipped");
    return SP_OK;
}

// ------------------------------------------------------------ Monte Carlo
// Colours of a graph by DSATUR (always the uncoloured vertex with the most
// distinct colours among its neighbours, ties to the higher degree, then
// the lower index; it takes the smallest colour free there).  Returns the
// number of colours.
int dsatur(const std::vector<std::vector<int>>& adj, std::vector<int>& col) {
    const int n = (int)adj.size();
    col.assign(n, -1);
    std::vector<std::set<int>> seen(n);
    int ncol = 0;
    for (int step = 0; step < n; ++step) {
        int v = -1;
        for (int u = 0; u < n; ++u) {
            if (col[u] >= 0) continue;
            if (v < 0 || seen[u].size() > seen[v].size() ||
                (seen[u].size() == seen[v].size() && adj[u].size() > adj[v].size()))
                v = u;
        }
        int c = 0;
        while (seen[v].count(c)) ++c;
        col[v] = c;
        ncol = std::max(ncol, c + 1);
        for (int u : adj[v]) seen[u].insert(c);
    }
    return ncol;
}

// Periodic colouring of the sites for the Metropolis sweep: site
// (a, b, c, beta) takes colour col[((a mod ma) mb + b mod mb) mc + c mod mc][beta],
// with periods 1-6 per axis (dividing the length of a periodic axis) such
// that no bond joins two sites of one colour: the quotient graph of the
// bonds on the ma x mb x mc x n_basis classes must have no loop, and is
// coloured by DSATUR; the periods giving the fewest colours win (ties to
// the smaller period product).
int mc_plan(sp_engine* e) {
    const HostGeo& g = e->geo;
    if (e->ham.ddi) return fail(e, SP_E_UNSUPPORTED, "Monte Carlo sweeps do not support the dipole term");
    std::vector<int> cand[3];
    for (int k = 0; k < 3; ++k)
        for (int m = 1; m <= 6; ++m)
            if (m <= g.n[k] && (!g.per[k] || g.n[k] % m == 0)) cand[k].push_back(m);
    int best = 1 << 30, best_prod = 1 << 30;
    for (int ma : cand[0])
        for (int mb : cand[1])
            for (int mc : cand[2]) {
                const int cells = ma * mb * mc, nodes = cells * g.nb;
                std::vector<std::vector<int>> adj(nodes);
                bool ok = true;
                for (int ia = 0; ia < ma && ok; ++ia)
                    for (int ib = 0; ib < mb && ok; ++ib)
                        for (int ic = 0; ic < mc && ok; ++ic)
                            for (int beta = 0; beta < g.nb && ok; ++beta) {
                                const int u = ((ia * mb + ib) * mc + ic) * g.nb + beta;
                                for (int q = e->bstart[beta]; q < e->bstart[beta + 1]; ++q) {
                                    const HostBond& b = e->bonds[q];
                                    const int ja = ((ia + b.d[0]) % ma + ma) % ma;
                                    const int jb = ((ib + b.d[1]) % mb + mb) % mb;
                                    const int jc = ((ic + b.d[2]) % mc + mc) % mc;
                                    const int v = ((ja * mb + jb) * mc + jc) * g.nb + b.bj;
                                    if (v == u) {
                                        ok = false;
                                        break;
                                    }
                                    adj[u].push_back(v);
                                    adj[v].push_back(u);
                                }
                            }
                if (!ok) continue;
                std::vector<int> col;
                const int K = dsatur(adj, col);
                if (K < best || (K == best && cells < best_prod)) {
                    best = K;
                    best_prod = cells;
                    e->mc_m[0] = ma;
                    e->mc_m[1] = mb;
                    e->mc_m[2] = mc;
                    e->mc_col.assign(col.begin(), col.end());
                }
            }
    if (best == (1 << 30))
        return fail(e, SP_E_UNSUPPORTED,
                    "no periodic colouring with periods up to 6 keeps bonded sites apart (lattice too short?)");
    e->mc_ncol = best;
    return SP_OK;
}

template <typename T>
int mc_run_impl(sp_engine* e, const sp_mc_params* p, int64_t n_sweeps, int64_t observe_every, sp_observation* obs,
                int64_t* accepted, double* cone_out) {
    const int64_t n_obs = observe_every > 0 ? n_sweeps / observe_every : 0;
    int rc;
    if (n_obs > e->obs_cap) {
        if ((rc = dalloc(e, e->d_obs, (size_t)n_obs * sp::OBS_NVALS * sizeof(double)))) return rc;
        e->obs_cap = n_obs;
    }
    const unsigned blocks = blocks_for(e->N);
    unsigned int* acc = nullptr;
    if ((rc = dalloc(e, acc, blocks * sizeof(unsigned int) + e->mc_col.size()))) return rc;
    HIPCHK(e, hipMemsetAsync(acc, 0, blocks * sizeof(unsigned int), e->stream));
    // the colour table rides behind the acceptance counts
    unsigned char* col = reinterpret_cast<unsigned char*>(acc + blocks);
    HIPCHK(e, hipMemcpyAsync(col, e->mc_col.data(), e->mc_col.size(), hipMemcpyHostToDevice, e->stream));
    const sp::Lattice L = make_lattice(e);
    // decisions in FP64 for every engine precision: FP64 couplings
    const sp::BondCoef<double> C = make_coef64(e);
    const sp::Phys<double> P = make_phys<double>(e, nullptr);
    sp::McArgs<double> M{};
    M.col = col;
    for (int q = 0; q < 3; ++q) M.cm[q] = e->mc_m[q];
    M.kT = kKB * p->T_K;
    M.cos_cone = std::cos(p->cone_deg * M_PI / 180.0);
    double* state = nullptr;   // adaptive cone: (cone, accepted count at the previous sweep)
    const bool adaptive = p->target_acceptance > 0.0;
    if (adaptive) {
        if ((rc = dalloc(e, state, 2 * sizeof(double)))) { dfree(*reinterpret_cast<void**>(&acc)); return rc; }
        const double init[2] = {p->cone_deg, 0.0};
        HIPCHK(e, hipMemcpyAsync(state, init, sizeof(init), hipMemcpyHostToDevice, e->stream));
        HIPCHK(e, hipStreamSynchronize(e->stream));
        M.cone_dev = state;
    }
    M.key.seed_lo = (uint32_t)p->seed;
    M.key.seed_hi = (uint32_t)(p->seed >> 32);
    M.key.replica = p->replica;
    int64_t k = 0;
    for (int64_t t = 0; t < n_sweeps; ++t) {
        M.key.step_lo = (uint32_t)e->step;
        M.key.step_hi = (uint32_t)(e->step >> 32);
        for (int colour = 0; colour < e->mc_ncol; ++colour) {
            M.colour = colour;
            hipLaunchKernelGGL((sp::k_mc_colour<T>), dim3(blocks), dim3(256), 0, e->stream, L, C, P, M,
                               static_cast<T*>(e->d_n), acc);
        }
        if (adaptive)
            hipLaunchKernelGGL(sp::k_mc_adapt, dim3(1), dim3(256), 0, e->stream, acc, (int)blocks, (long long)e->N,
                               p->target_acceptance, state);
        ++e->step;
        if (observe_every > 0 && (t + 1) % observe_every == 0) {
            rc = launch_observe<T>(e, e->d_n, e->d_obs + k * sp::OBS_NVALS, (long long)e->step, false);
            if (rc) {
                dfree(*reinterpret_cast<void**>(&acc));
                dfree(*reinterpret_cast<void**>(&state));
                return rc;
            }
            ++k;
        }
    }
    hipError_t st = hipGetLastError();
    std::vector<unsigned int> h(blocks);
    if (st == hipSuccess) st = hipMemcpyAsync(h.data(), acc, blocks * sizeof(unsigned int), hipMemcpyDeviceToHost, e->stream);
    std::vector<double> ho((size_t)n_obs * sp::OBS_NVALS);
    if (st == hipSuccess && n_obs > 0 && obs)
        st = hipMemcpyAsync(ho.data(), e->d_obs, ho.size() * sizeof(double), hipMemcpyDeviceToHost, e->stream);
    double fin[2] = {p->cone_deg, 0.0};
    if (st == hipSuccess && adaptive)
        st = hipMemcpyAsync(fin, state, sizeof(fin), hipMemcpyDeviceToHost, e->stream);
    if (st == hipSuccess) st = hipStreamSynchronize(e->stream);
    dfree(*reinterpret_cast<void**>(&acc));
    dfree(*reinterpret_cast<void**>(&state));
    if (cone_out) *cone_out = fin[0];
    if (st != hipSuccess) return fail(e, SP_E_HIP, std::string("Monte Carlo run: ") + hipGetErrorString(st));
    if (accepted) {
        int64_t s = 0;
        for (unsigned int v : h) s += v;
        *accepted = s;
    }
    if (n_obs > 0 && obs) {
        const int64_t step0 = (int64_t)e->step - n_sweeps;
        for (int64_t q = 0; q < n_obs; ++q)
            obs_from(&ho[(size_t)q * sp::OBS_NVALS], step0 + (q + 1) * observe_every, e->N, &obs[q]);
    }
    return SP_OK;
}

}  // namespace

namespace {
int install_ham(sp_engine* e, const HostHam& H, const std::vector<HostBond>& bonds, const std::vector<int>& bstart,
                const std::vector<HostBond>& all_bonds, bool explicit_pairs);
}  // namespace

#define DISPATCH(e, fn, ...) ((e)->precision == SP_F64 ? fn<double>(__VA_ARGS__) : fn<float>(__VA_ARGS__))

extern "C" {

const char* sp_version(void) { return kVersion; }

int sp_create(sp_engine** out, int device, int precision, void* hip_stream) {
    if (!out) return SP_E_ARG;
    *out = nullptr;
    if (precision != SP_F32 && precision != SP_F64) return SP_E_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SP_E_HIP;
    sp_engine* e = new (std::nothrow) sp_engine();
    if (!e) return SP_E_NOMEM;
    e->device = device;
    e->precision = precision;
    if (hipSetDevice(device) != hipSuccess) { delete e; return SP_E_HIP; }
    (void)scratch_for_device(device);
    if (hip_stream) {
        e->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess) { delete e; return SP_E_HIP; }
        e->own_stream = true;
    }
    if (dalloc(e, e->d_flag, sizeof(int)) || dalloc(e, e->d_abort_step, sizeof(long long)) ||
        dalloc(e, e->d_pstatus, sizeof(int)) || dalloc(e, e->d_step, sizeof(unsigned long long)) ||
        dalloc(e, e->d_obs_index, sizeof(long long)) || dalloc(e, e->d_obs_stage, sp::OBS_NVALS * sizeof(double)) ||
        hipHostMalloc((void**)&e->h_pin, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        sp_destroy(e);
        return SP_E_NOMEM;
    }
    (void)hipMemset(e->d_flag, 0, sizeof(int));
    *out = e;
    return SP_OK;
}

void sp_destroy(sp_engine* e) {
    if (!e) return;
    (void)hipSetDevice(e->device);
    // Wait for the engine's own work only: its stream if it owns one; a
    // borrowed stream may already be gone, so then the device is drained.
    // The flag lines of the persistent path go first, before any other
    // buffer the last launch touched.
    if (e->own_stream && e->stream)
        (void)hipStreamSynchronize(e->stream);
    else
        (void)hipDeviceSynchronize();
    dfree(*reinterpret_cast<void**>(&e->d_pflags));
    dfree(*reinterpret_cast<void**>(&e->d_pstatus));
    free_state_buffers(e);
    dfree(*reinterpret_cast<void**>(&e->d_partials));
    dfree(*reinterpret_cast<void**>(&e->d_obs));
    dfree(*reinterpret_cast<void**>(&e->d_flag));
    dfree(*reinterpret_cast<void**>(&e->d_abort_step));
    dfree(*reinterpret_cast<void**>(&e->d_step));
    dfree(*reinterpret_cast<void**>(&e->d_obs_index));
    dfree(*reinterpret_cast<void**>(&e->d_obs_stage));
    if (e->h_pin) (void)hipHostFree(e->h_pin);
    surrogate_free(e->sur);
    if (e->own_stream && e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

const char* sp_last_error(const sp_engine* e) { return e ? e->err.c_str() : "null engine"; }

int sp_mc_run(sp_engine* e, const sp_mc_params* p, int64_t n_sweeps, int64_t observe_every, sp_observation* obs,
              int64_t* accepted, double* cone_out) {
    int rc = check_ready(e, true);
    if (rc) return rc;
    if (!p) return fail(e, SP_E_ARG, "Monte Carlo params are NULL");
    if (!(p->T_K > 0.0) || !std::isfinite(p->T_K)) return fail(e, SP_E_ARG, "T must be finite and > 0");
    if (!(p->cone_deg > 0.0) || !(p->cone_deg <= 180.0)) return fail(e, SP_E_ARG, "cone angle must be in (0, 180]");
    if (!(p->target_acceptance >= 0.0 && p->target_acceptance < 1.0))
        return fail(e, SP_E_ARG, "target acceptance must be in [0, 1)");
    if (n_sweeps < 0 || observe_every < 0) return fail(e, SP_E_ARG, "n_sweeps and observe_every must be >= 0");
    if (observe_every > 0 && n_sweeps / observe_every > 0 && !obs) return fail(e, SP_E_ARG, "obs is NULL");
    if ((rc = mc_plan(e))) return rc;
    (void)hipSetDevice(e->device);
    if (cone_out) *cone_out = p->cone_deg;
    return DISPATCH(e, mc_run_impl, e, p, n_sweeps, observe_every, obs, accepted, cone_out);
}

int sp_set_geometry(sp_engine* e, const double bravais[9], int n_basis, const double* basis, const int n_cells[3],
                    const int periodic[3], double lattice_constant) {
    if (!e) return SP_E_ARG;
    if (!bravais || !basis || !n_cells || !periodic) return fail(e, SP_E_ARG, "null geometry argument");
    if (n_basis < 1 || n_basis > SP_MAX_BASIS) return fail(e, SP_E_ARG, "n_basis must be in 1..8");
    if (!(lattice_constant > 0.0) || !std::isfinite(lattice_constant))
        return fail(e, SP_E_ARG, "lattice constant must be finite and > 0");
    long long N = (long long)n_basis;
    for (int k = 0; k < 3; ++k) {
        if (n_cells[k] < 1) return fail(e, SP_E_ARG, "n_cells must be >= 1");
        if (periodic[k] != 0 && periodic[k] != 1) return fail(e, SP_E_ARG, "periodic flags must be 0 or 1");
        N *= n_cells[k];
    }
    if (N > (1LL << 29)) return fail(e, SP_E_UNSUPPORTED, "more than 2^29 sites");
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(bravais[k])) return fail(e, SP_E_ARG, "non-finite Bravais vector");
    double det = bravais[0] * (bravais[4] * bravais[8] - bravais[5] * bravais[7]) -
                 bravais[1] * (bravais[3] * bravais[8] - bravais[5] * bravais[6]) +
                 bravais[2] * (bravais[3] * bravais[7] - bravais[4] * bravais[6]);
    if (!(std::fabs(det) > 1e-12)) return fail(e, SP_E_ARG, "Bravais vectors are linearly dependent");
    HostGeo g{};
    std::memcpy(g.bravais, bravais, 9 * sizeof(double));
    g.nb = n_basis;
    for (int k = 0; k < 3 * n_basis; ++k) {
        if (!std::isfinite(basis[k])) return fail(e, SP_E_ARG, "non-finite basis position");
        g.basis[k] = basis[k];
    }
    for (int k = 0; k < 3; ++k) {
        g.n[k] = n_cells[k];
        g.per[k] = periodic[k];
    }
    g.a = lattice_constant;
    (void)hipSetDevice(e->device);
    free_state_buffers(e);
    e->geo = g;
    e->N = (int)N;
    e->has_geo = true;
    e->has_ham = false;
    e->has_spins = false;
    e->path = "none";
    e->step = 0;
    return SP_OK;
}

int sp_set_hamiltonian(sp_engine* e, const sp_hamiltonian* h) {
    if (!e) return SP_E_ARG;
    if (!e->has_geo) return fail(e, SP_E_ORDER, "sp_set_geometry has not been called");
    if (!h) return fail(e, SP_E_ARG, "null Hamiltonian");
    if (h->n_basis != e->geo.nb) return fail(e, SP_E_ARG, "n_basis differs from the geometry");
    if (!h->mu) return fail(e, SP_E_ARG, "mu is NULL");
    if (h->n_exch_shells < 0 || h->n_exch_shells > SP_MAX_SHELLS || h->n_dmi_shells < 0 ||
        h->n_dmi_shells > SP_MAX_SHELLS)
        return fail(e, SP_E_ARG, "shell counts must be in 0..8");
    if ((h->n_exch_shells > 0 && !h->J) || (h->n_dmi_shells > 0 && !h->D))
        return fail(e, SP_E_ARG, "J or D array is NULL");
    if (h->n_dmi_shells > 0 && h->dmi_kind != SP_DMI_BULK && h->dmi_kind != SP_DMI_INTERFACIAL)
        return fail(e, SP_E_ARG, "dmi_kind must be SP_DMI_BULK or SP_DMI_INTERFACIAL");
    if (h->n_gauss < 0 || h->n_gauss > SP_MAX_GAUSS) return fail(e, SP_E_ARG, "n_gauss must be in 0..16");
    if (h->n_gauss > 0 && (!h->gauss_a || !h->gauss_sigma || !h->gauss_c))
        return fail(e, SP_E_ARG, "Gaussian parameter arrays are NULL");
    if (h->ddi_mode != SP_DDI_OFF && h->ddi_mode != SP_DDI_DIRECT && h->ddi_mode != SP_DDI_SURROGATE &&
        h->ddi_mode != SP_DDI_FFT)
        return fail(e, SP_E_UNSUPPORTED, "ddi_mode must be SP_DDI_OFF, SP_DDI_DIRECT, SP_DDI_SURROGATE or SP_DDI_FFT");
    HostHam H{};
    for (int b = 0; b < e->geo.nb; ++b) {
        if (!(h->mu[b] > 0.0) || !std::isfinite(h->mu[b])) return fail(e, SP_E_ARG, "mu must be finite and > 0");
        H.mu[b] = h->mu[b];
        H.K[b] = h->K ? h->K[b] : 0.0;
        if (!std::isfinite(H.K[b])) return fail(e, SP_E_ARG, "non-finite K");
        double ax[3] = {0.0, 0.0, 1.0};
        if (h->K_axis) {
            for (int k = 0; k < 3; ++k) ax[k] = h->K_axis[3 * b + k];
        } else if (h->K && H.K[b] != 0.0) {
            return fail(e, SP_E_ARG, "K_axis is NULL but K is non-zero");
        }
        const double nrm = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) return fail(e, SP_E_ARG, "anisotropy axis has zero length");
        for (int k = 0; k < 3; ++k) H.Kax[3 * b + k] = ax[k] / nrm;
    }
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(h->B[k])) return fail(e, SP_E_ARG, "non-finite B");
        H.B[k] = h->B[k];
    }
    H.n_exch = h->n_exch_shells;
    H.n_dmi = h->n_dmi_shells;
    for (int s = 0; s < H.n_exch; ++s) H.J[s] = h->J[s];
    for (int s = 0; s < H.n_dmi; ++s) H.D[s] = h->D[s];
    H.dmi_kind = h->n_dmi_shells > 0 ? h->dmi_kind : SP_DMI_INTERFACIAL;
    H.ddi = h->ddi_mode;   // off, direct sum, surrogate (with direct-sum fallback), FFT convolution
    H.n_gauss = h->n_gauss;
    for (int k = 0; k < H.n_gauss; ++k) {
        const double* c = h->gauss_c + 3 * k;
        const double r = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (!(h->gauss_sigma[k] > 0.0) || !std::isfinite(h->gauss_sigma[k]) || !std::isfinite(h->gauss_a[k]) ||
            !(r > 0.0) || !std::isfinite(r))
            return fail(e, SP_E_ARG, "Gaussian potentials need sigma > 0, finite a and a non-zero centre");
        H.ga[k] = h->gauss_a[k];
        H.gsigma[k] = h->gauss_sigma[k];
        for (int q = 0; q < 3; ++q) H.gc[3 * k + q] = c[q] / r;
    }

    std::vector<HostBond> bonds, all_bonds;
    std::vector<int> bstart;
    int rc = build_bonds(e, e->geo, H, bonds, bstart, all_bonds);
    if (rc) return rc;
    return install_ham(e, H, bonds, bstart, all_bonds, false);
}

}  // extern "C"

namespace {

// Installs a Hamiltonian and its bond table (shell-built or explicit pairs):
// device buffers, bond upload, step-path selection; spins are kept.
int install_ham(sp_engine* e, const HostHam& H, const std::vector<HostBond>& bonds, const std::vector<int>& bstart,
                const std::vector<HostBond>& all_bonds, bool explicit_pairs) {
    int rc;
    // checks that can fail without a device error come before any state is replaced
    if (H.ddi == SP_DDI_FFT && (rc = fft_check(e))) return rc;
    (void)hipSetDevice(e->device);
    // keep spins across a Hamiltonian change only if already uploaded
    const bool had_spins = e->has_spins;
    std::vector<double> saved;
    if (had_spins) {
        saved.resize(3 * (size_t)e->N);
        if ((rc = DISPATCH(e, copy_out_soa, e, saved.data(), e->d_n, 3LL * e->N))) return rc;
    }
    free_state_buffers(e);
    e->ham = H;
    e->bonds = bonds;
    e->all_bonds = all_bonds;
    e->explicit_pairs = explicit_pairs;
    e->n_shells = explicit_pairs ? 0 : std::max(H.n_exch, H.n_dmi);
    e->bstart = bstart;
    e->R = 0;
    e->planar = true;
    for (const HostBond& b : bonds) {
        e->R = std::max(e->R, std::max(std::abs(b.d[0]), std::abs(b.d[1])));
        if (b.d[2] != 0) e->planar = false;
    }
    const size_t vbytes = 3 * (size_t)e->N * e->esz();
    if ((rc = dalloc(e, e->d_n, vbytes)) || (rc = dalloc(e, e->d_n2, vbytes)) || (rc = dalloc(e, e->d_np, vbytes)) ||
        (rc = dalloc(e, e->d_A, vbytes)) || (rc = dalloc(e, e->d_g, vbytes))) {
        free_state_buffers(e);
        e->has_ham = false;
        e->has_spins = false;
        return rc;
    }
    if (H.ddi) {
        const int tiles = (e->N + 255) / 256;
        e->dd_slices = std::max(1, std::min(16, (2048 * 256 * 2) / std::max(e->N, 1)));
        e->dd_slices = std::min(e->dd_slices, tiles);
        if ((rc = dalloc(e, e->d_gdd, vbytes)) || (rc = dalloc(e, e->d_gddp, vbytes)) ||
            (rc = dalloc(e, e->d_ddpart, vbytes * e->dd_slices))) {
            free_state_buffers(e);
            e->has_ham = false;
            e->has_spins = false;
            return rc;
        }
    }
    if ((rc = DISPATCH(e, upload_ham, e)) || (H.ddi == SP_DDI_FFT && (rc = DISPATCH(e, fft_setup, e)))) {
        free_state_buffers(e);
        e->has_ham = false;
        e->has_spins = false;
        return rc;
    }
    const int rows = (int)std::min<long long>(1024, (e->N + 255) / 256);
    if (rows > e->partial_rows) {
        if ((rc = dalloc(e, e->d_partials, (size_t)rows * sp::OBS_NVALS * sizeof(double)))) return rc;
    }
    e->partial_rows = rows;
    e->has_ham = true;

    // step path
    const HostGeo& g = e->geo;
    bool fused = g.nb == 1 && g.n[2] == 1 && e->planar && !H.ddi && H.n_gauss == 0 && e->R <= 2 &&
                 (int)bonds.size() <= sp::kMaxStencil;
    if (g.per[0] && g.n[0] <= 2 * e->R) fused = false;
    if (g.per[1] && g.n[1] <= 2 * e->R) fused = false;
    e->fused_ok = fused;
    e->tile_ok = !fused && tile_fits(e, H);
    e->path = fused ? "fused2d" : e->tile_ok ? "fusedtile" : "twopass";
    // compile-time stencil: the bond table must match a known shape, DMI may
    // sit on the first shell only, and every DMI vector must be in-plane
    e->shape = -1;
    e->shape_ndmi = 0;
    // default tile: 64x16 sites, one site per thread (fastest measured on the
    // 512^2 triangular workload); FP64 has a single configuration
    e->tile_cfg = e->precision == SP_F64 ? 0 : 4;
    if (fused && !explicit_pairs) {
        bool ok = true;
        for (const HostBond& b : all_bonds)
            if (b.D[2] != 0.0 || (b.shell > 0 && (b.D[0] != 0.0 || b.D[1] != 0.0))) ok = false;
        const int shp = ok ? detect_shape(e) : -1;
        if (shp >= 0) {
            e->shape = shp;
            for (const HostBond& b : all_bonds)
                if (b.shell == 0 && (b.D[0] != 0.0 || b.D[1] != 0.0)) e->shape_ndmi = 1;
            e->path = "shape2d";
        }
    }
    // 3D one-atom lattices: streamed fused path when the bond table matches a
    // compile-time simple-cubic stencil (DMI on the first shell only)
    e->shape3 = -1;
    e->shape3_ndmi = 0;
    e->shape3_dk = sp::DK_NONE;
    // default 3D tile: 32x32 columns, one 1024-thread workgroup per CU
    // (fastest measured on the 128^3 workload: 32.6 us against 33.4 for
    // 32x16 at two workgroups per CU); FP64 takes 16x16 (LDS)
    e->tile3_cfg = e->precision == SP_F64 ? 1 : 5;
    if (g.nb == 1 && g.n[2] > 1 && !H.ddi && H.n_gauss == 0 && !explicit_pairs) {
        bool ok = true;
        for (const HostBond& b : all_bonds)
            if (b.shell > 0 && (b.D[0] != 0.0 || b.D[1] != 0.0 || b.D[2] != 0.0)) ok = false;
        const int shp = ok ? detect_shape3(e) : -1;
        if (shp >= 0) {
            e->shape3 = shp;
            for (const HostBond& b : all_bonds)
                if (b.shell == 0 && (b.D[0] != 0.0 || b.D[1] != 0.0 || b.D[2] != 0.0)) e->shape3_ndmi = 1;
            e->shape3_dk = e->shape3_ndmi ? (bulk_dmi3(all_bonds, nullptr) ? sp::DK_BULK : sp::DK_GENERAL)
                                          : sp::DK_NONE;
            e->path = "shape3d";
        }
    }
    e->path_label = e->path;
    if (e->shape >= 0) e->path_label += std::string("/") + kTileCfgs[e->tile_cfg].name;
    if (e->shape3 >= 0) e->path_label += std::string("/") + kTile3Cfgs[e->tile3_cfg].name;

    if (had_spins) {
        if ((rc = DISPATCH(e, copy_in_soa, e, e->d_n, saved.data(), 3LL * e->N))) return rc;
        e->has_spins = true;
    }
    return SP_OK;
}

constexpr int kMaxPairOffset = 64;       // |dcell| per axis in sp_set_pairs
constexpr int kMaxBondsPerBasis = 256;   // directed bonds per basis atom

}  // namespace

extern "C" {

int sp_set_pairs(sp_engine* e, int64_t n_pairs, const int* bi, const int* bj, const int* dcell, const double* J,
                 const double* D) {
    int rc = check_ready(e, false);
    if (rc) return rc;
    if (n_pairs < 0) return fail(e, SP_E_ARG, "n_pairs must be >= 0");
    if (n_pairs > 0 && (!bi || !bj || !dcell || !J)) return fail(e, SP_E_ARG, "pair arrays are NULL");
    const int nb = e->geo.nb;
    std::vector<std::vector<HostBond>> per(nb);
    std::set<std::array<int, 5>> seen;
    for (int64_t p = 0; p < n_pairs; ++p) {
        const std::string at = "pair " + std::to_string(p) + ": ";
        if (bi[p] < 0 || bi[p] >= nb || bj[p] < 0 || bj[p] >= nb) return fail(e, SP_E_ARG, at + "basis index out of range");
        const int* d = dcell + 3 * p;
        for (int k = 0; k < 3; ++k)
            if (d[k] < -kMaxPairOffset || d[k] > kMaxPairOffset)
                return fail(e, SP_E_ARG, at + "cell offset beyond +-" + std::to_string(kMaxPairOffset));
        if (bi[p] == bj[p] && d[0] == 0 && d[1] == 0 && d[2] == 0) return fail(e, SP_E_ARG, at + "a spin paired with itself");
        HostBond f{};
        f.bi = bi[p];
        f.bj = bj[p];
        f.shell = -1;
        f.J = J[p];
        for (int k = 0; k < 3; ++k) {
            f.d[k] = d[k];
            f.D[k] = D ? D[3 * p + k] : 0.0;
        }
        if (!std::isfinite(f.J) || !std::isfinite(f.D[0]) || !std::isfinite(f.D[1]) || !std::isfinite(f.D[2]))
            return fail(e, SP_E_ARG, at + "non-finite J or D");
        const std::array<int, 5> key{f.bi, f.bj, d[0], d[1], d[2]}, rkey{f.bj, f.bi, -d[0], -d[1], -d[2]};
        if (seen.count(key) || seen.count(rkey)) return fail(e, SP_E_ARG, at + "repeats an earlier pair or its reverse");
        seen.insert(key);
        // the same pair seen from j: n_j x n_i = -(n_i x n_j), so D changes sign
        HostBond r = f;
        r.bi = f.bj;
        r.bj = f.bi;
        for (int k = 0; k < 3; ++k) {
            r.d[k] = -d[k];
            r.D[k] = -f.D[k];
        }
        per[f.bi].push_back(f);
        per[r.bi].push_back(r);
        if ((int)per[f.bi].size() > kMaxBondsPerBasis || (int)per[r.bi].size() > kMaxBondsPerBasis)
            return fail(e, SP_E_ARG, "more than " + std::to_string(kMaxBondsPerBasis) + " bonds on one basis atom");
    }
    std::vector<HostBond> bonds;
    std::vector<int> bstart(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        bstart[b] = (int)bonds.size();
        for (const HostBond& q : per[b])
            if (q.J != 0.0 || q.D[0] != 0.0 || q.D[1] != 0.0 || q.D[2] != 0.0) bonds.push_back(q);
    }
    bstart[nb] = (int)bonds.size();
    HostHam H = e->ham;
    H.n_exch = 0;   // the shells no longer define the pair terms
    H.n_dmi = 0;
    return install_ham(e, H, bonds, bstart, bonds, true);
}

int64_t sp_num_sites(const sp_engine* e) { return e && e->has_geo ? e->N : 0; }

int sp_get_bonds(sp_engine* e, int beta, double* out, int max_bonds) {
    if (!e) return SP_E_ARG;
    int rc = check_ready(e, false);
    if (rc) return rc;
    if (beta < 0 || beta >= e->geo.nb) return fail(e, SP_E_ARG, "basis index out of range");
    int k = 0;
    for (const HostBond& b : e->bonds) {
        if (b.bi != beta) continue;
        if (out && k < max_bonds) {
            double* o = out + 10 * k;
            o[0] = b.bj; o[1] = b.d[0]; o[2] = b.d[1]; o[3] = b.d[2]; o[4] = b.shell;
            o[5] = b.J; o[6] = b.D[0]; o[7] = b.D[1]; o[8] = b.D[2]; o[9] = 0.0;
        }
        ++k;
    }
    return k;
}

int sp_set_spins(sp_engine* e, const double* n_soa, int64_t N) {
    int rc = check_ready(e, false);
    if (rc) return rc;
    if (!n_soa || N != e->N) return fail(e, SP_E_ARG, "spin array size differs from the number of sites");
    std::vector<double> v(3 * (size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        const double x = n_soa[i], y = n_soa[N + i], z = n_soa[2 * N + i];
        const double r = std::sqrt(x * x + y * y + z * z);
        if (!(r > 0.0) || !std::isfinite(r))
            return fail(e, SP_E_ARG, "spin " + std::to_string(i) + " has zero or non-finite length");
        v[i] = x / r;
        v[N + i] = y / r;
        v[2 * N + i] = z / r;
    }
    (void)hipSetDevice(e->device);
    if ((rc = DISPATCH(e, copy_in_soa, e, e->d_n, v.data(), 3 * N))) return rc;
    e->has_spins = true;
    return SP_OK;
}

int sp_get_spins(sp_engine* e, double* n_soa, int64_t N) {
    int rc = check_ready(e, true);
    if (rc) return rc;
    if (!n_soa || N != e->N) return fail(e, SP_E_ARG, "spin array size differs from the number of sites");
    (void)hipSetDevice(e->device);
    return DISPATCH(e, copy_out_soa, e, n_soa, e->d_n, 3 * N);
}

int sp_set_spins_dev(sp_engine* e, const void* n_soa_dev, int64_t N) {
    int rc = check_ready(e, false);
    if (rc) return rc;
    if (!n_soa_dev || N != e->N) return fail(e, SP_E_ARG, "spin array size differs from the number of sites");
    (void)hipSetDevice(e->device);
    HIPCHK(e, hipMemcpyAsync(e->d_n, n_soa_dev, 3 * (size_t)N * e->esz(), hipMemcpyDeviceToDevice, e->stream));
    e->has_spins = true;
    return SP_OK;
}

int sp_get_spins_dev(sp_engine* e, void* n_soa_dev, int64_t N) {
    int rc = check_ready(e, true);
    if (rc) return rc;
    if (!n_soa_dev || N != e->N) return fail(e, SP_E_ARG, "spin array size differs from the number of sites");
    (void)hipSetDevice(e->device);
    HIPCHK(e, hipMemcpyAsync(n_soa_dev, e->d_n, 3 * (size_t)N * e->esz(), hipMemcpyDeviceToDevice, e->stream));
    return SP_OK;
}

int sp_set_step(sp_engine* e, uint64_t step) {
    if (!e) return SP_E_ARG;
    e->step = step;
    return SP_OK;
}

uint64_t sp_get_step(const sp_engine* e) { return e ? e->step : 0; }

int sp_gradient_dev(sp_engine* e, void* g_soa_dev, int64_t N) {
    int rc = check_ready(e, true);
    if (rc) return rc;
    if (!g_soa_dev || N != e->N) return fail(e, SP_E_ARG, "gradient array size differs from the number of sites");
    (void)hipSetDevice(e->device);
    return DISPATCH(e, gradient_dev, e, e->d_n, g_soa_dev);
}

int sp_gradient(sp_engine* e, double* g_soa, int64_t N) {
    int rc = check_ready(e, true);
    if (rc) return rc;
    if (!g_soa || N != e->N) return fail(e, SP_E_ARG, "gradient array size differs from the number of sites");
    (void)hipSetDevice(e->device);
    if ((rc = DISPATCH(e, gradient_dev, e, e->d_n, e->d_g))) return rc;
    return DISPATCH(e, copy_out_soa, e, g_soa, e->d_g, 3 * N);
}

int sp_observe(sp_engine* e, sp_observation* obs) {
    int rc = check_ready(e, true);
    if (rc) return rc;
    if (!obs) return fail(e, SP_E_ARG, "observation pointer is NULL");
    (void)hipSetDevice(e->device);
    double* d_out = nullptr;
    if ((rc = dalloc(e, d_out, sp::OBS_NVALS * sizeof(double)))) return rc;
    rc = DISPATCH(e, launch_observe, e, e->d_n, d_out, (long long)e->step, false);
    if (rc == SP_OK) {
        hipError_t s = hipMemcpyAsync(e->h_pin, d_out, sp::OBS_NVALS * sizeof(double), hipMemcpyDeviceToHost, e->stream);
        if (s == hipSuccess) s = hipStreamSynchronize(e->stream);
        if (s != hipSuccess) rc = fail(e, SP_E_HIP, hipGetErrorString(s));
        else obs_from(e->h_pin, (int64_t)e->step, e->N, obs);
    }
    void* p = d_out;
    dfree(p);
    return rc;
}

int sp_energy(sp_engine* e, double* E_total, double per_term[5]) {
    sp_observation o{};
    int rc = sp_observe(e, &o);
    if (rc) return rc;
    if (E_total) *E_total = o.E;
    if (per_term)
        for (int k = 0; k < 5; ++k) per_term[k] = o.per_term[k];
    return SP_OK;
}

int sp_llg_step(sp_engine* e, const sp_llg_params* p) {
    int rc = check_ready(e, true);
    if (rc) return rc;
    if ((rc = check_llg(e, p))) return rc;
    (void)hipSetDevice(e->device);
    HIPCHK(e, hipMemsetAsync(e->d_flag, 0, sizeof(int), e->stream));
    if ((rc = DISPATCH(e, launch_step, e, p, e->step, e->d_n, e->d_n2))) return rc;
    std::swap(e->d_n, e->d_n2);
    ++e->step;
    return SP_OK;
}

int sp_run(sp_engine* e, const sp_llg_params* p, int64_t n_steps, int64_t observe_every, sp_observation* obs) {
    int rc = check_ready(e, true);
    if (rc) return rc;
    if ((rc = check_llg(e, p))) return rc;
    if (n_steps < 0 || observe_every < 0) return fail(e, SP_E_ARG, "n_steps and observe_every must be >= 0");
    (void)hipSetDevice(e->device);
    return DISPATCH(e, run_impl, e, p, n_steps, observe_every, 0.0, obs, nullptr);
}

int sp_run_tol(sp_engine* e, const sp_llg_params* p, int64_t max_steps, int64_t observe_every, double tol,
               sp_observation* obs, int64_t* steps_done) {
    if (steps_done) *steps_done = 0;
    int rc = check_ready(e, true);
    if (rc) return rc;
    if ((rc = check_llg(e, p))) return rc;
    if (max_steps < 0 || observe_every <= 0) return fail(e, SP_E_ARG, "max_steps must be >= 0, observe_every > 0");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(e, SP_E_ARG, "tol must be finite and > 0");
    (void)hipSetDevice(e->device);
    return DISPATCH(e, run_impl, e, p, max_steps, observe_every, tol, obs, steps_done);
}

int sp_set_graph_replay(sp_engine* e, int enable) {
    if (!e) return SP_E_ARG;
    e->graphs_on = enable != 0;
    if (!e->graphs_on) drop_graphs(e);
    return SP_OK;
}

int sp_synchronize(sp_engine* e) {
    if (!e) return SP_E_ARG;
    HIPCHK(e, hipStreamSynchronize(e->stream));
    return SP_OK;
}

int sp_dipole_gradient_dev(sp_engine* e, const void* n_soa_dev, void* g_soa_dev, int64_t N) {
    int rc = check_ready(e, false);
    if (rc) return rc;
    if (!n_soa_dev || !g_soa_dev || N != e->N) return fail(e, SP_E_ARG, "array size differs from the number of sites");
    if (!e->ham.ddi) return fail(e, SP_E_ORDER, "the Hamiltonian has no dipole term (ddi_mode off)");
    (void)hipSetDevice(e->device);
    return DISPATCH(e, launch_dipole, e, n_soa_dev, g_soa_dev);
}

int sp_dipole_gradient_dev_noalloc(sp_engine* e, const void* n_soa_dev, void* g_soa_dev, int64_t N) {
    int rc = check_ready(e, false);
    if (rc) return rc;
    if (!n_soa_dev || !g_soa_dev || N != e->N) return fail(e, SP_E_ARG, "array size differs from the number of sites");
    if (!e->ham.ddi) return fail(e, SP_E_ORDER, "the Hamiltonian has no dipole term (ddi_mode off)");
    const size_t need = 3 * (size_t)e->N * e->esz() * (size_t)e->dd_slices;
    if (need > kScratchBytes)
        return fail(e, SP_E_ARG, "the direct sum of " + std::to_string(e->N) + " sites needs " + std::to_string(need) +
                                     " bytes of partial sums; the static scratch holds " +
                                     std::to_string(kScratchBytes));
    (void)hipSetDevice(e->device);
    void* part = scratch_for_device(e->device);
    if (!part) return fail(e, SP_E_HIP, "hipGetSymbolAddress of the static scratch failed on this device");
    return DISPATCH(e, launch_direct_sum_into, e, n_soa_dev, g_soa_dev, part);
}

int sp_dipole_gradient(sp_engine* e, double* g_soa, int64_t N) {
    int rc = check_ready(e, true);
    if (rc) return rc;
    if (!g_soa || N != e->N) return fail(e, SP_E_ARG, "array size differs from the number of sites");
    if (!e->ham.ddi) return fail(e, SP_E_ORDER, "the Hamiltonian has no dipole term (ddi_mode off)");
    (void)hipSetDevice(e->device);
    if ((rc = DISPATCH(e, launch_dipole, e, e->d_n, e->d_g))) return rc;
    return DISPATCH(e, copy_out_soa, e, g_soa, e->d_g, 3 * N);
}

int sp_thermal_normals(sp_engine* e, uint64_t seed, uint64_t step, uint32_t replica, uint32_t site0, int64_t n_sites,
                       double* eta_soa, uint32_t* raw4) {
    if (!e) return SP_E_ARG;
    if (!eta_soa || n_sites <= 0 || n_sites > (1LL << 26)) return fail(e, SP_E_ARG, "bad normals request");
    (void)hipSetDevice(e->device);
    return DISPATCH(e, normals_dev, e, seed, step, replica, site0, n_sites, eta_soa, raw4);
}

const char* sp_step_path(const sp_engine* e) { return e ? e->path_label.c_str() : "none"; }

int sp_set_step_path(sp_engine* e, const char* name) {
    int rc = check_ready(e, false);
    if (rc) return rc;
    if (!name) return fail(e, SP_E_ARG, "path name is NULL");
    const std::string s(name);
    if (s == "twopass") {
        e->path = "twopass";
    } else if (s == "fused2d") {
        if (!e->fused_ok) return fail(e, SP_E_UNSUPPORTED, "fused2d needs a one-atom 2D lattice without dipole");
        e->path = "fused2d";
    } else if (s == "fusedtile") {
        if (!e->tile_ok)
            return fail(e, SP_E_UNSUPPORTED,
                        "fusedtile needs 2-4 atoms per cell in 2D (reach <= 2) or 1-3 (FP64: 1-2) in 3D (reach <= 1), "
                        "no dipole or Gaussian terms");
        e->path = "fusedtile";
    } else if (s.rfind("shape2d", 0) == 0) {
        if (e->shape < 0)
            return fail(e, SP_E_UNSUPPORTED, "shape2d needs a bond table matching a compile-time stencil");
        int cfg = 0;
        if (s.size() > 7) {
            if (s[7] != '/') return fail(e, SP_E_ARG, "unknown step path " + s);
            cfg = -1;
            const int ncfg = e->precision == SP_F64 ? kNumTileCfgsF64 : kNumTileCfgs;
            for (int k = 0; k < ncfg; ++k)
                if (s.substr(8) == kTileCfgs[k].name) cfg = k;
            if (cfg < 0) return fail(e, SP_E_ARG, "unknown tile configuration in " + s);
        }
        e->path = "shape2d";
        e->tile_cfg = cfg;
    } else if (s.rfind("shape3d", 0) == 0) {
        if (e->shape3 < 0)
            return fail(e, SP_E_UNSUPPORTED, "shape3d needs a 3D one-atom bond table matching a compile-time stencil");
        int cfg = e->precision == SP_F64 ? 1 : 5;
        if (s.size() > 7) {
            if (s[7] != '/') return fail(e, SP_E_ARG, "unknown step path " + s);
            cfg = -1;
            for (int k = 0; k < kNumTile3Cfgs; ++k)
                if (s.substr(8) == kTile3Cfgs[k].name && (e->precision != SP_F64 || k == 1 || k == 3)) cfg = k;
            if (cfg < 0) return fail(e, SP_E_ARG, "unknown tile configuration in " + s);
        }
        e->path = "shape3d";
        e->tile3_cfg = cfg;
    } else if (s.rfind("persist2d", 0) == 0) {
        int cfg = e->precision == SP_F64 ? 2 : 0;
        if (s.size() > 9) {
            if (s[9] != '/') return fail(e, SP_E_ARG, "unknown step path " + s);
            cfg = -1;
            for (int k = 0; k < kNumPersistCfgs; ++k)
                if (s.substr(10) == kPersistCfgs[k].name && (e->precision != SP_F64 || kPersistCfgs[k].f64)) cfg = k;
            if (cfg < 0) return fail(e, SP_E_ARG, "unknown tile configuration in " + s);
        }
        const int keep = e->persist_cfg;
        e->persist_cfg = cfg;
        sp_llg_params probe{};
        probe.alpha = 0.1;
        probe.dt_ps = 1e-3;
        rc = e->precision == SP_F64 ? launch_persist<double>(e, &probe, 1, true)
                                    : launch_persist<float>(e, &probe, 1, true);
        if (rc) {
            e->persist_cfg = keep;
            return rc;
        }
        e->path = "persist2d";
        e->tile_cfg = kPersistCfgs[cfg].tile_cfg;
    } else {
        return fail(e, SP_E_ARG, "unknown step path " + s);
    }
    e->path_label = e->path;
    if (std::strcmp(e->path, "shape2d") == 0) e->path_label += std::string("/") + kTileCfgs[e->tile_cfg].name;
    if (std::strcmp(e->path, "shape3d") == 0) e->path_label += std::string("/") + kTile3Cfgs[e->tile3_cfg].name;
    if (std::strcmp(e->path, "persist2d") == 0) e->path_label += std::string("/") + kPersistCfgs[e->persist_cfg].name;
    return SP_OK;
}

int sp_autotune(sp_engine* e, const sp_llg_params* p, int n_steps, double* ms_per_step) {
    int rc = check_ready(e, true);
    if (rc) return rc;
    if ((rc = check_llg(e, p))) return rc;
    if (n_steps < 1 || n_steps > 100000) return fail(e, SP_E_ARG, "n_steps must be in 1..100000");
    (void)hipSetDevice(e->device);
    std::vector<std::string> cands{"twopass"};
    if (e->tile_ok) cands.push_back("fusedtile");
    if (e->shape3 >= 0)
        for (int k = 0; k < kNumTile3Cfgs; ++k)
            if (e->precision != SP_F64 || k == 1 || k == 3) cands.push_back(std::string("shape3d/") + kTile3Cfgs[k].name);
    if (p->solver != SP_SOLVER_DEPONDT) {
        // Heun and SIB: the two-pass kernels, the fused tile or the one tile shape they are built for
        if (e->shape >= 0)
            cands.push_back(std::string("shape2d/") + (e->precision == SP_F64 ? kSolverTileF64 : kSolverTileF32));
    } else {
        if (e->fused_ok) cands.push_back("fused2d");

        if (e->shape >= 0) {
            const int ncfg = e->precision == SP_F64 ? kNumTileCfgsF64 : kNumTileCfgs;
            for (int k = 0; k < ncfg; ++k) cands.push_back(std::string("shape2d/") + kTileCfgs[k].name);
            const int keep_cfg = e->persist_cfg;
            const std::string keep_err = e->err;
            for (int k = 0; k < kNumPersistCfgs; ++k) {
                if (e->precision == SP_F64 && !kPersistCfgs[k].f64) continue;
                e->persist_cfg = k;
                const int ok = e->precision == SP_F64 ? launch_persist<double>(e, p, 1, true)
                                                      : launch_persist<float>(e, p, 1, true);
                if (ok == SP_OK) cands.push_back(std::string("persist2d/") + kPersistCfgs[k].name);
            }
            e->persist_cfg = keep_cfg;
            e->err = keep_err;
        }
    }
    const std::string keep_label = e->path_label;
    const uint64_t keep_step = e->step;
    const size_t bytes = 3 * (size_t)e->N * e->esz();
    void* backup = nullptr;
    if ((rc = dalloc(e, backup, bytes))) return rc;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    double best = 1e300;
    std::string best_name = keep_label;
    int out = SP_OK;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess ||
        hipMemcpyAsync(backup, e->d_n, bytes, hipMemcpyDeviceToDevice, e->stream) != hipSuccess) {
        out = fail(e, SP_E_HIP, "autotune set-up failed");
    }
    for (size_t c = 0; out == SP_OK && c < cands.size(); ++c) {
        if ((rc = sp_set_step_path(e, cands[c].c_str()))) { out = rc; break; }
        float ms = 0.0f;
        const bool pers = std::strcmp(e->path, "persist2d") == 0 && p->solver == SP_SOLVER_DEPONDT;
        if (pers) {
            // warm-up launch, then all n_steps in one launch
            e->step = keep_step;
            rc = hipMemsetAsync(e->d_pstatus, 0, sizeof(int), e->stream) == hipSuccess ? SP_OK : SP_E_HIP;
            if (!rc) rc = DISPATCH(e, launch_persist, e, p, 1, false);
            if (!rc && hipEventRecord(t0, e->stream) != hipSuccess) rc = SP_E_HIP;
            if (!rc) rc = DISPATCH(e, launch_persist, e, p, n_steps, false);
        } else {
            // warm-up (code load, caches), then the timed steps
            rc = DISPATCH(e, launch_step, e, p, e->step, e->d_n, e->d_n2);
            if (!rc && hipEventRecord(t0, e->stream) != hipSuccess) rc = SP_E_HIP;
            for (int k = 0; !rc && k < n_steps; ++k) {
                rc = DISPATCH(e, launch_step, e, p, keep_step + k, (k & 1) ? e->d_n2 : e->d_n,
                              (k & 1) ? e->d_n : e->d_n2);
            }
        }
        if (!rc && (hipEventRecord(t1, e->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                    hipEventElapsedTime(&ms, t0, t1) != hipSuccess))
            rc = SP_E_HIP;
        if (!rc && pers) {
            int pst = 0;
            if (hipMemcpy(&pst, e->d_pstatus, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess || pst) rc = SP_E_HIP;
            if (pst) e->pgen = (1u << 30) + 1;
        }
        if (!rc && hipMemcpyAsync(e->d_n, backup, bytes, hipMemcpyDeviceToDevice, e->stream) != hipSuccess)
            rc = SP_E_HIP;
        if (rc) { out = rc == SP_E_HIP ? fail(e, SP_E_HIP, "autotune timing failed") : rc; break; }
        if (ms / n_steps < best) {
            best = ms / n_steps;
            best_name = cands[c];
        }
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipStreamSynchronize(e->stream);
    dfree(backup);
    e->step = keep_step;
    const int rc2 = sp_set_step_path(e, out == SP_OK ? best_name.c_str() : keep_label.c_str());
    if (out == SP_OK && ms_per_step) *ms_per_step = best;
    return out != SP_OK ? out : rc2;
}

}  // extern "C"

// ====================================================================== batch
namespace {

constexpr TileCfg kBatchCfgs[] = {{"32x16x512", 32, 16, 512}, {"64x16x1024", 64, 16, 1024}};
constexpr int kNumBatchCfgs = 2;

struct BatchRep {
    int na, nb, per_a, per_b;
    sp_llg_params p;
    int resident;        // 0 tiled, 32 or 64: resident replica side
    size_t off;          // offset (floats) of buffer 0 in the arena; buffer 1 follows
    std::vector<float> init;
};

}  // namespace

struct sp_gneb {
    sp_engine* e = nullptr;
    int device = 0;
    int M = 0, N = 0, nblk = 0;
    double k = 1.0, dt = 0.1, m = 1.0;
    void *x = nullptr, *v = nullptr, *F = nullptr, *Fp = nullptr, *g = nullptr, *tau = nullptr;
    double* part = nullptr;  // force partials (v.F, F.F)
    double* epart = nullptr; // energy partials [M][nblk]
    double* tpart = nullptr; // tangent partials [M][nblk][3]
    double* E = nullptr;    // [M]
    double* s3 = nullptr;   // [3M]: |tau|^2, g.tau, l^2
    double* vf = nullptr;   // [2]
    int* types = nullptr;   // [M] image types (0 normal, 1 climbing, 2 falling)
    double* fmax = nullptr; // [(M-2) nblk] block maxima of |F_i|^2 (convergence test)
    int* stop = nullptr;    // [2]: converged flag, iteration that passed
    int64_t iterations = 0;
    sp_batch* batch = nullptr;   // the batch that advances the chain, if attached
    std::string err;
};

struct sp_batch {
    int device = 0;
    hipStream_t stream = nullptr, side = nullptr;
    bool own_stream = false;
    std::string err;
    bool has_template = false;
    HostHam ham{};
    std::vector<HostBond> all_bonds;
    int n_shells = 0, shape = -1, shape_ndmi = 0;
    sp::ShapeCoef<float> C{};
    sp::StepCoef<float> SC{};   // the tiled replicas' step kernel (as the single-engine step)
    sp::Site2D<float> Q{};
    std::vector<BatchRep> reps;
    bool finalized = false;
    float* arena = nullptr;
    size_t arena_floats = 0;
    sp::ReplicaDesc<float>* d_reps = nullptr;
    int2* d_work = nullptr;
    int n_work = 0;
    int* d_res32 = nullptr;
    int* d_res64 = nullptr;
    int n_res32 = 0, n_res64 = 0;
    unsigned long long* d_step = nullptr;
    uint64_t step = 0;
    int parity = 0;
    int cfg = 0;
    int chunk = 32;
    hipGraphExec_t gexec = nullptr;
    hipGraphExec_t gexec_chain = nullptr;     // an attached chain's chunk, launched beside gexec
    int g_parity = -1, g_cfg = -1, g_chunk = -1;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    sp_gneb* gneb = nullptr;                   // attached GNEB chain (FP32), advanced by every run
    hipStream_t gside = nullptr;               // its branch of the chunk graph
    hipEvent_t ev_gfork = nullptr, ev_gjoin = nullptr;
};

namespace {

template <typename T>
int gneb_enqueue(sp_gneb* G, int n_iter, hipStream_t st, double tol = 0.0);

int bfail(sp_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    return code;
}

#define BHIPCHK(b, call)                                                                      \
    do {                                                                                      \
        hipError_t _s = (call);                                                               \
        if (_s != hipSuccess)                                                                 \
            return bfail((b), SP_E_HIP, std::string(#call) + ": " + hipGetErrorString(_s));   \
    } while (0)

bool same_ham(const HostHam& a, const HostHam& b) {
    return std::memcmp(&a, &b, sizeof(HostHam)) == 0;
}

// Drop the captured chunk graphs (they no longer match the batch).
void batch_drop_graphs(sp_batch* b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->gexec_chain) (void)hipGraphExecDestroy(b->gexec_chain);
    b->gexec = nullptr;
    b->gexec_chain = nullptr;
}

int batch_build_work(sp_batch* b) {
    const TileCfg& tc = kBatchCfgs[b->cfg];
    std::vector<sp::ReplicaDesc<float>> desc(b->reps.size());
    std::vector<int2> work;
    std::vector<int> r32, r64;
    for (size_t r = 0; r < b->reps.size(); ++r) {
        const BatchRep& R = b->reps[r];
        sp::ReplicaDesc<float>& D = desc[r];
        D.n[0] = b->arena + R.off;
        D.n[1] = b->arena + R.off + 3 * (size_t)R.na * R.nb;
        D.na = R.na;
        D.nb = R.nb;
        D.per_a = R.per_a;
        D.per_b = R.per_b;
        D.tiles_x = (R.na + tc.TX - 1) / tc.TX;
        D.thermal = R.p.T_K > 0.0 ? 1 : 0;
        const double mm = b->ham.mu[0] * kMuB;
        D.sigma = R.p.T_K > 0.0 ? (float)std::sqrt(2.0 * R.p.alpha * kKB * R.p.T_K / (kGamma * mm * R.p.dt_ps)) : 0.0f;
        D.gp = (float)(kGamma / (1.0 + R.p.alpha * R.p.alpha));
        D.alpha = (float)R.p.alpha;
        D.dt = (float)R.p.dt_ps;
        D.seed_lo = (uint32_t)R.p.seed;
        D.seed_hi = (uint32_t)(R.p.seed >> 32);
        D.replica = R.p.replica;
        if (R.resident == 32) {
            r32.push_back((int)r);
        } else if (R.resident == 64) {
            r64.push_back((int)r);
        } else {
            const int tiles_y = (R.nb + tc.TY - 1) / tc.TY;
            for (int t = 0; t < D.tiles_x * tiles_y; ++t) work.push_back(make_int2((int)r, t));
        }
    }
    void* p = b->d_reps; dfree(p); b->d_reps = nullptr;
    p = b->d_work; dfree(p); b->d_work = nullptr;
    p = b->d_res32; dfree(p); b->d_res32 = nullptr;
    p = b->d_res64; dfree(p); b->d_res64 = nullptr;
    auto up = [&](auto*& dst, const void* src, size_t bytes) -> int {
        void* q = nullptr;
        if (bytes == 0) return SP_OK;
        if (hipMalloc(&q, bytes) != hipSuccess) return bfail(b, SP_E_NOMEM, "batch table allocation failed");
        if (hipMemcpy(q, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
            return bfail(b, SP_E_HIP, "batch table upload failed");
        dst = static_cast<std::remove_reference_t<decltype(dst)>>(q);
        return SP_OK;
    };
    int rc;
    if ((rc = up(b->d_reps, desc.data(), desc.size() * sizeof(desc[0])))) return rc;
    if ((rc = up(b->d_work, work.data(), work.size() * sizeof(int2)))) return rc;
    if ((rc = up(b->d_res32, r32.data(), r32.size() * sizeof(int)))) return rc;
    if ((rc = up(b->d_res64, r64.data(), r64.size() * sizeof(int)))) return rc;
    b->n_work = (int)work.size();
    b->n_res32 = (int)r32.size();
    b->n_res64 = (int)r64.size();
    batch_drop_graphs(b);
    return SP_OK;
}

int batch_finalize(sp_batch* b) {
    if (b->finalized) return SP_OK;
    if (b->reps.empty()) return bfail(b, SP_E_ORDER, "the batch has no replicas");
    size_t total = 0;
    for (BatchRep& R : b->reps) {
        R.off = total;
        total += 6 * (size_t)R.na * R.nb;
    }
    void* q = nullptr;
    if (hipMalloc(&q, total * sizeof(float)) != hipSuccess) return bfail(b, SP_E_NOMEM, "batch arena allocation failed");
    b->arena = static_cast<float*>(q);
    b->arena_floats = total;
    for (BatchRep& R : b->reps) {
        BHIPCHK(b, hipMemcpy(b->arena + R.off, R.init.data(), R.init.size() * sizeof(float), hipMemcpyHostToDevice));
        std::vector<float>().swap(R.init);
    }
    if (hipMalloc(&q, sizeof(unsigned long long)) != hipSuccess) return bfail(b, SP_E_NOMEM, "allocation failed");
    b->d_step = static_cast<unsigned long long*>(q);
    const unsigned long long s0 = b->step;
    BHIPCHK(b, hipMemcpy(b->d_step, &s0, sizeof(s0), hipMemcpyHostToDevice));
    int rc = batch_build_work(b);
    if (rc) return rc;
    b->finalized = true;
    return SP_OK;
}

template <int S, int NDMI>
void batch_launch_resident(sp_batch* b, hipStream_t s, int n_steps) {
    if (b->n_res32)
        hipLaunchKernelGGL((sp::k_batch_resident<float, S, NDMI, 32, 32, 1024>), dim3(b->n_res32), dim3(1024), 0, s,
                           b->C, b->Q, b->d_reps, b->d_res32, b->d_step, n_steps);
    if (b->n_res64)
        hipLaunchKernelGGL((sp::k_batch_resident<float, S, NDMI, 64, 64, 1024>), dim3(b->n_res64), dim3(1024), 0, s,
                           b->C, b->Q, b->d_reps, b->d_res64, b->d_step, n_steps);
}

template <int S, int NDMI>
void batch_launch_tiled(sp_batch* b, hipStream_t s, int k, int parity) {
    if (!b->n_work) return;
    if (b->cfg == 1)
        hipLaunchKernelGGL((sp::k_batch_tiled<float, S, NDMI, 64, 16, 1024>), dim3(b->n_work), dim3(1024), 0, s, b->SC,
                           b->Q, b->d_reps, b->d_work, b->d_step, k, parity);
    else
        hipLaunchKernelGGL((sp::k_batch_tiled<float, S, NDMI, 32, 16, 512>), dim3(b->n_work), dim3(512), 0, s, b->SC,
                           b->Q, b->d_reps, b->d_work, b->d_step, k, parity);
}

template <int S>
void batch_chunk_shape(sp_batch* b, int n_steps, int parity, bool with_chain) {
    // resident replicas on the side stream, tiled steps on the main stream
    (void)hipEventRecord(b->ev_fork, b->stream);
    (void)hipStreamWaitEvent(b->side, b->ev_fork, 0);
    if (b->shape_ndmi) batch_launch_resident<S, sp::ShapeTab<S>::NB0>(b, b->side, n_steps);
    else batch_launch_resident<S, 0>(b, b->side, n_steps);
    // an attached GNEB chain: n_steps iterations on a third branch (unless
    // the caller launches the chain's own graph beside this chunk's)
    const bool chain = with_chain && b->gneb;
    if (chain) {
        (void)hipEventRecord(b->ev_gfork, b->stream);
        (void)hipStreamWaitEvent(b->gside, b->ev_gfork, 0);
        (void)gneb_enqueue<float>(b->gneb, n_steps, b->gside);
    }
    for (int k = 0; k < n_steps; ++k) {
        if (b->shape_ndmi) batch_launch_tiled<S, sp::ShapeTab<S>::NB0>(b, b->stream, k, parity);
        else batch_launch_tiled<S, 0>(b, b->stream, k, parity);
    }
    (void)hipEventRecord(b->ev_join, b->side);
    (void)hipStreamWaitEvent(b->stream, b->ev_join, 0);
    if (chain) {
        (void)hipEventRecord(b->ev_gjoin, b->gside);
        (void)hipStreamWaitEvent(b->stream, b->ev_gjoin, 0);
    }
    hipLaunchKernelGGL(sp::k_advance_step, dim3(1), dim3(64), 0, b->stream, b->d_step, n_steps);
}

// Enqueue one chunk of n_steps on b->stream (also used under graph capture).
void batch_chunk(sp_batch* b, int n_steps, int parity, bool with_chain = true) {
    switch (b->shape) {
        case sp::SH_SQ1: batch_chunk_shape<sp::SH_SQ1>(b, n_steps, parity, with_chain); break;
        case sp::SH_SQ2: batch_chunk_shape<sp::SH_SQ2>(b, n_steps, parity, with_chain); break;
        case sp::SH_SQ3: batch_chunk_shape<sp::SH_SQ3>(b, n_steps, parity, with_chain); break;
        case sp::SH_TRI1: batch_chunk_shape<sp::SH_TRI1>(b, n_steps, parity, with_chain); break;
        case sp::SH_TRI2: batch_chunk_shape<sp::SH_TRI2>(b, n_steps, parity, with_chain); break;
        default: batch_chunk_shape<sp::SH_TRI3>(b, n_steps, parity, with_chain); break;
    }
}

// The chunk as graphs: the replicas' (resident and tiled branches, then the
// step counter), and an attached chain's chunk of iterations as a graph of
// its own.  Launched on two streams, the chain's graph runs beside the
// replicas'; branches inside one graph were measured to run one after the
// other.
int batch_capture(sp_batch* b) {
    batch_drop_graphs(b);
    hipGraph_t g = nullptr;
    BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    batch_chunk(b, b->chunk, b->parity, false);
    hipError_t s = hipStreamEndCapture(b->stream, &g);
    if (s != hipSuccess) return bfail(b, SP_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(s));
    s = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (s != hipSuccess) return bfail(b, SP_E_HIP, std::string("graph instantiation failed: ") + hipGetErrorString(s));
    if (b->gneb) {
        BHIPCHK(b, hipStreamBeginCapture(b->gside, hipStreamCaptureModeThreadLocal));
        (void)gneb_enqueue<float>(b->gneb, b->chunk, b->gside);
        s = hipStreamEndCapture(b->gside, &g);
        if (s != hipSuccess) return bfail(b, SP_E_HIP, std::string("chain graph capture failed: ") + hipGetErrorString(s));
        s = hipGraphInstantiate(&b->gexec_chain, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (s != hipSuccess)
            return bfail(b, SP_E_HIP, std::string("chain graph instantiation failed: ") + hipGetErrorString(s));
    }
    b->g_parity = b->parity;
    b->g_cfg = b->cfg;
    b->g_chunk = b->chunk;
    return SP_OK;
}

int batch_advance(sp_batch* b, int64_t n_steps, bool use_graph) {
    int64_t left = n_steps;
    while (use_graph && left >= b->chunk) {
        if (!b->gexec || b->g_parity != b->parity || b->g_cfg != b->cfg || b->g_chunk != b->chunk ||
            (b->gneb != nullptr) != (b->gexec_chain != nullptr)) {
            int rc = batch_capture(b);
            if (rc) return rc;
        }
        if (b->gexec_chain) {   // the chain's chunk beside the replicas', joined before the next chunk
            BHIPCHK(b, hipEventRecord(b->ev_gfork, b->stream));
            BHIPCHK(b, hipStreamWaitEvent(b->gside, b->ev_gfork, 0));
            BHIPCHK(b, hipGraphLaunch(b->gexec_chain, b->gside));
        }
        BHIPCHK(b, hipGraphLaunch(b->gexec, b->stream));
        if (b->gexec_chain) {
            BHIPCHK(b, hipEventRecord(b->ev_gjoin, b->gside));
            BHIPCHK(b, hipStreamWaitEvent(b->stream, b->ev_gjoin, 0));
        }
        left -= b->chunk;
    }
    while (left > 0) {
        const int k = (int)std::min<int64_t>(left, 1024);
        batch_chunk(b, k, b->parity);
        BHIPCHK(b, hipGetLastError());
        b->parity ^= (k & 1);
        left -= k;
    }
    b->step += (uint64_t)n_steps;
    if (b->gneb) b->gneb->iterations += n_steps;
    return SP_OK;
}

}  // namespace

extern "C" {

int sp_batch_create(sp_batch** out, int device, void* hip_stream) {
    if (!out) return SP_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SP_E_HIP;
    sp_batch* b = new (std::nothrow) sp_batch();
    if (!b) return SP_E_NOMEM;
    b->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete b; return SP_E_HIP; }
    if (hip_stream) {
        b->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) { delete b; return SP_E_HIP; }
        b->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess) {
        sp_batch_destroy(b);
        return SP_E_HIP;
    }
    *out = b;
    return SP_OK;
}

void sp_batch_destroy(sp_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();   // the main stream may be borrowed and already gone
    batch_drop_graphs(b);
    void* p = b->arena; dfree(p);
    p = b->d_reps; dfree(p);
    p = b->d_work; dfree(p);
    p = b->d_res32; dfree(p);
    p = b->d_res64; dfree(p);
    p = b->d_step; dfree(p);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->gneb) b->gneb->batch = nullptr;   // the chain stays usable on its own
    if (b->ev_gfork) (void)hipEventDestroy(b->ev_gfork);
    if (b->ev_gjoin) (void)hipEventDestroy(b->ev_gjoin);
    if (b->gside) (void)hipStreamDestroy(b->gside);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char* sp_batch_last_error(const sp_batch* b) { return b ? b->err.c_str() : "null batch"; }

int sp_batch_add(sp_batch* b, sp_engine* e, const sp_llg_params* p) {
    if (!b || !e) return SP_E_ARG;
    if (b->finalized) return bfail(b, SP_E_ORDER, "replicas cannot be added after the first sp_batch_run");
    if (!e->has_geo || !e->has_ham || !e->has_spins) return bfail(b, SP_E_ORDER, "engine has no lattice or spins");
    if (e->precision != SP_F32) return bfail(b, SP_E_UNSUPPORTED, "batches are FP32");
    if (e->shape < 0) return bfail(b, SP_E_UNSUPPORTED, "replica lattice does not match a compile-time stencil");
    if (check_llg(e, p)) return bfail(b, SP_E_ARG, e->err);
    if (p->solver != SP_SOLVER_DEPONDT) return bfail(b, SP_E_UNSUPPORTED, "batches run Depondt's scheme only");
    if (!b->has_template) {
        b->ham = e->ham;
        b->all_bonds = e->all_bonds;
        b->n_shells = e->n_shells;
        b->shape = e->shape;
        b->shape_ndmi = e->shape_ndmi;
        switch (e->shape) {
            case sp::SH_SQ1: b->C = shape_coef_for<float, sp::SH_SQ1>(e); b->SC = step_coef_for<float, sp::SH_SQ1>(e); break;
            case sp::SH_SQ2: b->C = shape_coef_for<float, sp::SH_SQ2>(e); b->SC = step_coef_for<float, sp::SH_SQ2>(e); break;
            case sp::SH_SQ3: b->C = shape_coef_for<float, sp::SH_SQ3>(e); b->SC = step_coef_for<float, sp::SH_SQ3>(e); break;
            case sp::SH_TRI1: b->C = shape_coef_for<float, sp::SH_TRI1>(e); b->SC = step_coef_for<float, sp::SH_TRI1>(e); break;
            case sp::SH_TRI2: b->C = shape_coef_for<float, sp::SH_TRI2>(e); b->SC = step_coef_for<float, sp::SH_TRI2>(e); break;
            default: b->C = shape_coef_for<float, sp::SH_TRI3>(e); b->SC = step_coef_for<float, sp::SH_TRI3>(e); break;
        }
        b->Q = make_site2d<float>(e, nullptr);
        b->has_template = true;
    } else if (!same_ham(b->ham, e->ham) || b->shape != e->shape || b->shape_ndmi != e->shape_ndmi) {
        return bfail(b, SP_E_ARG, "every replica of a batch must have the same Hamiltonian and stencil");
    }
    BatchRep R{};
    R.na = e->geo.n[0];
    R.nb = e->geo.n[1];
    R.per_a = e->geo.per[0];
    R.per_b = e->geo.per[1];
    R.p = *p;
    R.resident = 0;
    if (R.na == R.nb && (R.na == 32 || R.na == 64)) R.resident = R.na;
    R.init.resize(6 * (size_t)e->N);
    (void)hipSetDevice(e->device);
    if (hipStreamSynchronize(e->stream) != hipSuccess ||
        hipMemcpy(R.init.data(), e->d_n, 3 * (size_t)e->N * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return bfail(b, SP_E_HIP, "copying the replica's spins failed");
    std::copy(R.init.begin(), R.init.begin() + 3 * (size_t)e->N, R.init.begin() + 3 * (size_t)e->N);
    b->reps.push_back(std::move(R));
    return (int)b->reps.size() - 1;
}

int sp_batch_add_gneb(sp_batch* b, sp_gneb* G) {
    if (!b || !G) return SP_E_ARG;
    if (b->gneb) return bfail(b, SP_E_ORDER, "the batch already advances a GNEB chain");
    if (G->batch) return bfail(b, SP_E_ORDER, "the chain is attached to another batch");
    if (G->e->precision != SP_F32) return bfail(b, SP_E_ARG, "batches run FP32: the chain's engine must be FP32");
    if (G->device != b->device) return bfail(b, SP_E_ARG, "the chain lives on another device");
    (void)hipSetDevice(b->device);
    if (!b->gside && (hipStreamCreateWithFlags(&b->gside, hipStreamNonBlocking) != hipSuccess ||
                      hipEventCreateWithFlags(&b->ev_gfork, hipEventDisableTiming) != hipSuccess ||
                      hipEventCreateWithFlags(&b->ev_gjoin, hipEventDisableTiming) != hipSuccess))
        return bfail(b, SP_E_HIP, "stream creation failed");
    // the chain's own pending work ends before the batch takes it over
    BHIPCHK(b, hipStreamSynchronize(G->e->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    batch_drop_graphs(b);   // the captured chunk no longer matches
    b->gneb = G;
    G->batch = b;
    return SP_OK;
}

int sp_batch_run(sp_batch* b, int64_t n_steps) {
    if (!b) return SP_E_ARG;
    if (n_steps < 0) return bfail(b, SP_E_ARG, "n_steps must be >= 0");
    (void)hipSetDevice(b->device);
    int rc = batch_finalize(b);
    if (rc) return rc;
    return batch_advance(b, n_steps, true);
}

int sp_batch_get_spins(sp_batch* b, int slot, double* n_soa, int64_t N) {
    if (!b) return SP_E_ARG;
    if (slot < 0 || slot >= (int)b->reps.size()) return bfail(b, SP_E_ARG, "replica slot out of range");
    const BatchRep& R = b->reps[slot];
    const int64_t n = (int64_t)R.na * R.nb;
    if (!n_soa || N != n) return bfail(b, SP_E_ARG, "spin array size differs from the replica's size");
    std::vector<float> tmp(3 * (size_t)n);
    if (!b->finalized) {
        std::copy(R.init.begin(), R.init.begin() + 3 * n, tmp.begin());
    } else {
        (void)hipSetDevice(b->device);
        BHIPCHK(b, hipStreamSynchronize(b->stream));
        const int buf = R.resident ? 0 : b->parity;
        BHIPCHK(b, hipMemcpy(tmp.data(), b->arena + R.off + (size_t)buf * 3 * n, 3 * n * sizeof(float),
                             hipMemcpyDeviceToHost));
    }
    for (int64_t k = 0; k < 3 * n; ++k) n_soa[k] = tmp[k];
    return SP_OK;
}

int sp_batch_replica_info(sp_batch* b, int slot, int64_t* n_sites, int* resident) {
    if (!b) return SP_E_ARG;
    if (slot < 0 || slot >= (int)b->reps.size()) return bfail(b, SP_E_ARG, "replica slot out of range");
    if (n_sites) *n_sites = (int64_t)b->reps[slot].na * b->reps[slot].nb;
    if (resident) *resident = b->reps[slot].resident ? 1 : 0;
    return SP_OK;
}

int sp_batch_set_chunk(sp_batch* b, int steps) {
    if (!b) return SP_E_ARG;
    if (steps < 2 || steps > 1024 || (steps & 1)) return bfail(b, SP_E_ARG, "chunk must be even and in 2..1024");
    b->chunk = steps;
    return SP_OK;
}

uint64_t sp_batch_get_step(const sp_batch* b) { return b ? b->step : 0; }

int sp_batch_autotune(sp_batch* b, int n_steps, double* ms_per_step) {
    if (!b) return SP_E_ARG;
    if (n_steps < 2 || n_steps > 1024 || (n_steps & 1)) return bfail(b, SP_E_ARG, "n_steps must be even, 2..1024");
    (void)hipSetDevice(b->device);
    int rc = batch_finalize(b);
    if (rc) return rc;
    void* backup = nullptr;
    if (hipMalloc(&backup, b->arena_floats * sizeof(float)) != hipSuccess)
        return bfail(b, SP_E_NOMEM, "autotune backup allocation failed");
    const uint64_t keep_step = b->step;
    const int keep_parity = b->parity;
    sp_gneb* const keep_gneb = b->gneb;   // an attached chain is neither timed nor advanced
    b->gneb = nullptr;
    double best = 1e300;
    int best_cfg = b->cfg;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int out = SP_OK;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess ||
        hipMemcpy(backup, b->arena, b->arena_floats * sizeof(float), hipMemcpyDeviceToDevice) != hipSuccess)
        out = bfail(b, SP_E_HIP, "autotune set-up failed");
    for (int c = 0; out == SP_OK && c < kNumBatchCfgs; ++c) {
        b->cfg = c;
        if ((out = batch_build_work(b))) break;
        float ms = 0.0f;
        batch_chunk(b, 2, b->parity);  // warm-up
        if (hipEventRecord(t0, b->stream) != hipSuccess) { out = SP_E_HIP; break; }
        batch_chunk(b, n_steps, b->parity);
        if (hipEventRecord(t1, b->stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
            hipEventElapsedTime(&ms, t0, t1) != hipSuccess) {
            out = bfail(b, SP_E_HIP, "autotune timing failed");
            break;
        }
        if (ms / n_steps < best) {
            best = ms / n_steps;
            best_cfg = c;
        }
        // restore replicas and the device step counter
        const unsigned long long s0 = keep_step;
        if (hipMemcpy(b->arena, backup, b->arena_floats * sizeof(float), hipMemcpyDeviceToDevice) != hipSuccess ||
            hipMemcpy(b->d_step, &s0, sizeof(s0), hipMemcpyHostToDevice) != hipSuccess) {
            out = bfail(b, SP_E_HIP, "autotune restore failed");
            break;
        }
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipFree(backup);
    b->step = keep_step;
    b->parity = keep_parity;
    b->gneb = keep_gneb;
    b->cfg = best_cfg;
    const int rc2 = batch_build_work(b);
    if (out == SP_OK && ms_per_step) *ms_per_step = best;
    return out != SP_OK ? out : rc2;
}

}  // extern "C"

// ======================================================================= GNEB

namespace {

int gfail(sp_gneb* G, int code, const std::string& msg) {
    if (G) G->err = msg;
    return code;
}

// Images on the stencil path whose sides divide into the 64 x 4 tiles of
// k_gneb_grad_shape (then tiles and site blocks coincide in number).
bool gneb_tiles(const sp_gneb* G) {
    const sp_engine* e = G->e;
    return e->shape >= 0 && !e->ham.ddi && e->ham.n_gauss == 0 && e->geo.n[0] % 64 == 0 && e->geo.n[1] % 4 == 0 &&
           (long long)(e->geo.n[0] / 64) * (e->geo.n[1] / 4) == G->nblk;
}

template <typename T, int S>
void gneb_grad_shape(sp_gneb* G, hipStream_t st, const int* stop) {
    sp_engine* e = G->e;
    const sp::GnebDims d{G->M, G->N, G->nblk};
    const sp::ShapeCoef<double> C = shape_coef_for<double, S>(e);
    const sp::Site2D<double> Q = make_site2d<double>(e, nullptr);
    const int tiles_x = e->geo.n[0] / 64;
    const T* x = static_cast<const T*>(G->x);
    T* g = static_cast<T*>(G->g);
    const dim3 grid((unsigned)G->nblk, (unsigned)G->M);
    if (e->shape_ndmi)
        hipLaunchKernelGGL((sp::k_gneb_grad_shape<T, S, sp::ShapeTab<S>::NB0>), grid, dim3(256), 0, st, d, C, Q,
                           tiles_x, x, g, G->epart, stop);
    else
        hipLaunchKernelGGL((sp::k_gneb_grad_shape<T, S, 0>), grid, dim3(256), 0, st, d, C, Q, tiles_x, x, g, G->epart, stop);
}

template <typename T>
int gneb_forces(sp_gneb* G, bool update_v, hipStream_t st, const int* stop = nullptr) {
    sp_engine* e = G->e;
    const sp::GnebDims d{G->M, G->N, G->nblk};
    T* x = static_cast<T*>(G->x);
    T* g = static_cast<T*>(G->g);
    T* tau = static_cast<T*>(G->tau);
    if (gneb_tiles(G)) {
        switch (e->shape) {
            case sp::SH_SQ1: gneb_grad_shape<T, sp::SH_SQ1>(G, st, stop); break;
            case sp::SH_SQ2: gneb_grad_shape<T, sp::SH_SQ2>(G, st, stop); break;
            case sp::SH_SQ3: gneb_grad_shape<T, sp::SH_SQ3>(G, st, stop); break;
            case sp::SH_TRI1: gneb_grad_shape<T, sp::SH_TRI1>(G, st, stop); break;
            case sp::SH_TRI2: gneb_grad_shape<T, sp::SH_TRI2>(G, st, stop); break;
            default: gneb_grad_shape<T, sp::SH_TRI3>(G, st, stop); break;
        }
    } else {
        hipLaunchKernelGGL((sp::k_gneb_grad<T>), dim3(G->nblk, G->M), dim3(256), 0, st, d, make_lattice(e),
                           make_coef64(e), make_phys<double>(e, nullptr), x, g, G->epart, stop);
    }
    hipLaunchKernelGGL((sp::k_gneb_tangent<T>), dim3(G->nblk, G->M), dim3(256), 0, st, d, x, g, G->epart, G->E, tau,
                       G->tpart, stop);
    hipLaunchKernelGGL((sp::k_gneb_force<T>), dim3(G->nblk, G->M - 2), dim3(256), 0, st, d, (T)G->k,
                       (T)(G->dt / (2.0 * G->m)), update_v ? 1 : 0, x, g, tau, G->tpart, G->s3, G->types,
                       static_cast<T*>(G->F), static_cast<const T*>(G->Fp), static_cast<T*>(G->v), G->part,
                       stop ? G->fmax : nullptr, stop);
    if (update_v)
        hipLaunchKernelGGL((sp::k_gneb_sum<2>), dim3(1), dim3(256), 0, st, G->part, (G->M - 2) * G->nblk, G->vf,
                           stop);
    hipError_t s = hipGetLastError();
    if (s != hipSuccess) return gfail(G, SP_E_HIP, hipGetErrorString(s));
    return SP_OK;
}

template <typename T>
int gneb_project(sp_gneb* G, hipStream_t st) {
    const sp::GnebDims d{G->M, G->N, G->nblk};
    hipLaunchKernelGGL((sp::k_gneb_project<T>), dim3(G->nblk, G->M - 2), dim3(256), 0, st, d, G->vf,
                       static_cast<T*>(G->v), static_cast<const T*>(G->F), static_cast<T*>(G->Fp));
    hipError_t s = hipGetLastError();
    if (s != hipSuccess) return gfail(G, SP_E_HIP, hipGetErrorString(s));
    return SP_OK;
}

// n_iter velocity-projection iterations enqueued on st (also under graph
// capture); the iteration counter is the caller's business.
// With tol > 0 every iteration ends with the convergence test (largest
// per-spin force of the interior images below tol); once it passes, the
// launches of the remaining iterations return at once, so the chain is the
// one whose forces passed, projected as after any run.
template <typename T>
int gneb_enqueue(sp_gneb* G, int n_iter, hipStream_t st, double tol) {
    const sp::GnebDims d{G->M, G->N, G->nblk};
    const int* stop = tol > 0.0 ? G->stop : nullptr;
    if (stop) hipLaunchKernelGGL(sp::k_gneb_clear_stop, dim3(1), dim3(64), 0, st, G->stop, G->stop + 1);
    // the projection of each iteration is applied by the next move; the
    // state between calls is always projected (v, F_prev final)
    for (int it = 0; it < n_iter; ++it) {
        hipLaunchKernelGGL((sp::k_gneb_move<T>), dim3(G->nblk, G->M - 2), dim3(256), 0, st, d, (T)G->dt,
                           (T)(G->dt * G->dt / (2.0 * G->m)), it > 0 ? 1 : 0, G->vf, static_cast<const T*>(G->F),
                           static_cast<T*>(G->x), static_cast<T*>(G->v), static_cast<T*>(G->Fp), stop);
        int rc = gneb_forces<T>(G, true, st, stop);
        if (rc) return rc;
        if (stop)
            hipLaunchKernelGGL(sp::k_gneb_converged, dim3(1), dim3(256), 0, st, G->fmax, (G->M - 2) * G->nblk,
                               tol * tol, G->stop, G->stop + 1, it);
    }
    if (n_iter > 0) return gneb_project<T>(G, st);
    return SP_OK;
}

template <typename T>
int gneb_iterate(sp_gneb* G, int n_iter) {
    int rc = gneb_enqueue<T>(G, n_iter, G->e->stream);
    if (rc == SP_OK) G->iterations += n_iter;
    return rc;
}

// The stream that orders the chain's work: the batch's when attached.
hipStream_t gneb_stream(const sp_gneb* G) { return G->batch ? G->batch->stream : G->e->stream; }

template <typename T>
int gneb_upload(sp_gneb* G, const double* chain) {
    const size_t L = (size_t)3 * G->N;
    std::vector<T> h((size_t)G->M * L);
    for (int im = 0; im < G->M; ++im)
        for (int i = 0; i < G->N; ++i) {
            const double* c = chain + im * L;
            const double x = c[i], y = c[G->N + i], z = c[2 * G->N + i];
            const double r = std::sqrt(x * x + y * y + z * z);
            if (!(r > 0.0) || !std::isfinite(r)) return gfail(G, SP_E_ARG, "chain has a zero or non-finite spin");
            h[im * L + i] = (T)(x / r);
            h[im * L + G->N + i] = (T)(y / r);
            h[im * L + 2 * G->N + i] = (T)(z / r);
        }
    if (hipMemcpy(G->x, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return gfail(G, SP_E_HIP, "chain upload failed");
    return SP_OK;
}

template <typename T>
int gneb_download(sp_gneb* G, const void* src, double* out, size_t count) {
    std::vector<T> h(count);
    if (hipStreamSynchronize(gneb_stream(G)) != hipSuccess ||
        hipMemcpy(h.data(), src, count * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess)
        return gfail(G, SP_E_HIP, "download failed");
    for (size_t k = 0; k < count; ++k) out[k] = (double)h[k];
    return SP_OK;
}

void gneb_free(sp_gneb* G) {
    void* ps[] = {G->x,  G->v,  G->F,  G->Fp, G->g,     G->tau,  G->part, G->epart,
                  G->tpart, G->E, G->s3, G->vf, G->types, G->fmax, G->stop};
    for (void* p : ps)
        if (p) (void)hipFree(p);
}

}  // namespace

extern "C" {

int sp_gneb_create(sp_gneb** out, sp_engine* e, int n_images, const double* chain, double k_spring, double vp_dt,
                   double vp_mass) {
    if (!out) return SP_E_ARG;
    *out = nullptr;
    int rc = check_ready(e, false);
    if (rc) return rc;
    if (e->ham.ddi) return fail(e, SP_E_UNSUPPORTED, "GNEB chains do not support the dipole term");
    if (n_images < 3 || n_images > 4096 || !chain) return fail(e, SP_E_ARG, "a chain needs 3..4096 images");
    if (!(vp_dt > 0.0) || !(vp_mass > 0.0) || !std::isfinite(k_spring) || !std::isfinite(vp_dt) ||
        !std::isfinite(vp_mass))
        return fail(e, SP_E_ARG, "VP time step and mass must be finite and > 0, spring constant finite");
    sp_gneb* G = new (std::nothrow) sp_gneb();
    if (!G) return SP_E_NOMEM;
    G->e = e;
    G->device = e->device;
    G->M = n_images;
    G->N = e->N;
    G->nblk = (e->N + 255) / 256;
    G->k = k_spring;
    G->dt = vp_dt;
    G->m = vp_mass;
    (void)hipSetDevice(e->device);
    const size_t vb = (size_t)G->M * 3 * G->N * e->esz();
    const size_t parts = (size_t)(G->M - 2) * G->nblk * 2;
    void** bufs[] = {&G->x, &G->v, &G->F, &G->Fp, &G->g, &G->tau};
    for (void** b : bufs)
        if (hipMalloc(b, vb) != hipSuccess) { gneb_free(G); delete G; return fail(e, SP_E_NOMEM, "GNEB allocation failed"); }
    if (hipMalloc((void**)&G->part, parts * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&G->epart, (size_t)G->M * G->nblk * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&G->tpart, (size_t)G->M * G->nblk * 3 * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&G->E, G->M * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&G->s3, 3 * G->M * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&G->vf, 2 * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&G->types, G->M * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&G->fmax, (size_t)(G->M - 2) * G->nblk * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&G->stop, 2 * sizeof(int)) != hipSuccess) {
        gneb_free(G);
        delete G;
        return fail(e, SP_E_NOMEM, "GNEB allocation failed");
    }
    if (hipMemset(G->v, 0, vb) != hipSuccess || hipMemset(G->F, 0, vb) != hipSuccess ||
        hipMemset(G->Fp, 0, vb) != hipSuccess || hipMemset(G->tau, 0, vb) != hipSuccess ||
        hipMemset(G->vf, 0, 2 * sizeof(double)) != hipSuccess || hipMemset(G->types, 0, G->M * sizeof(int)) != hipSuccess ||
        hipMemset(G->stop, 0, 2 * sizeof(int)) != hipSuccess) {
        gneb_free(G);
        delete G;
        return fail(e, SP_E_HIP, "GNEB initialisation failed");
    }
    rc = e->precision == SP_F64 ? gneb_upload<double>(G, chain) : gneb_upload<float>(G, chain);
    if (rc == SP_OK)
        rc = e->precision == SP_F64 ? gneb_forces<double>(G, false, e->stream) : gneb_forces<float>(G, false, e->stream);
    // v = 0 (vf = 0 gives a zero projection) and F_prev = F
    if (rc == SP_OK)
        rc = e->precision == SP_F64 ? gneb_project<double>(G, e->stream) : gneb_project<float>(G, e->stream);
    if (rc == SP_OK && hipStreamSynchronize(e->stream) != hipSuccess) rc = SP_E_HIP;
    if (rc) {
        e->err = G->err;
        gneb_free(G);
        delete G;
        return rc;
    }
    *out = G;
    return SP_OK;
}

void sp_gneb_destroy(sp_gneb* G) {
    if (!G) return;
    // The engine may already be gone (its stream too): only the device is used.
    (void)hipSetDevice(G->device);
    (void)hipDeviceSynchronize();
    if (G->batch) {   // detach: the batch's captured chunk launches this chain's kernels
        sp_batch* b = G->batch;
        b->gneb = nullptr;
        batch_drop_graphs(b);
    }
    gneb_free(G);
    delete G;
}

const char* sp_gneb_last_error(const sp_gneb* G) { return G ? G->err.c_str() : "null chain"; }

int sp_gneb_set_image_type(sp_gneb* G, int image, int type) {
    if (!G) return SP_E_ARG;
    if (image < 1 || image > G->M - 2) return gfail(G, SP_E_ARG, "only interior images have a type");
    if (type != SP_IMAGE_NORMAL && type != SP_IMAGE_CLIMBING && type != SP_IMAGE_FALLING)
        return gfail(G, SP_E_ARG, "type must be SP_IMAGE_NORMAL, SP_IMAGE_CLIMBING or SP_IMAGE_FALLING");
    (void)hipSetDevice(G->e->device);
    const hipStream_t st = gneb_stream(G);
    if (hipMemcpyAsync(G->types + image, &type, sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return gfail(G, SP_E_HIP, "image type upload failed");
    // the previous force kept by the minimiser is left as it is; the next
    // iteration forms the new force with the new type
    return SP_OK;
}

int sp_gneb_iterate(sp_gneb* G, int n_iter) {
    if (!G) return SP_E_ARG;
    if (n_iter < 0) return gfail(G, SP_E_ARG, "n_iter must be >= 0");
    if (G->batch) return gfail(G, SP_E_ORDER, "the chain is attached to a batch: sp_batch_run advances it");
    (void)hipSetDevice(G->e->device);
    const int rc = G->e->precision == SP_F64 ? gneb_iterate<double>(G, n_iter) : gneb_iterate<float>(G, n_iter);
    if (rc) return rc;
    if (hipStreamSynchronize(G->e->stream) != hipSuccess) return gfail(G, SP_E_HIP, "synchronisation failed");
    return SP_OK;
}

int sp_gneb_iterate_tol(sp_gneb* G, int max_iter, double tol, int* iters_done) {
    if (iters_done) *iters_done = 0;
    if (!G) return SP_E_ARG;
    if (max_iter < 0) return gfail(G, SP_E_ARG, "max_iter must be >= 0");
    if (!(tol > 0.0) || !std::isfinite(tol)) return gfail(G, SP_E_ARG, "tol must be finite and > 0");
    if (G->batch) return gfail(G, SP_E_ORDER, "the chain is attached to a batch: sp_batch_run advances it");
    (void)hipSetDevice(G->e->device);
    const int rc = G->e->precision == SP_F64 ? gneb_enqueue<double>(G, max_iter, G->e->stream, tol)
                                             : gneb_enqueue<float>(G, max_iter, G->e->stream, tol);
    if (rc) return rc;
    int st[2] = {0, -1};
    if (max_iter > 0 &&
        (hipMemcpyAsync(st, G->stop, sizeof(st), hipMemcpyDeviceToHost, G->e->stream) != hipSuccess ||
         hipStreamSynchronize(G->e->stream) != hipSuccess))
        return gfail(G, SP_E_HIP, "synchronisation failed");
    const int done = st[0] ? st[1] + 1 : max_iter;
    G->iterations += done;
    if (iters_done) *iters_done = done;
    return SP_OK;
}

int sp_gneb_get_chain(sp_gneb* G, double* chain) {
    if (!G || !chain) return SP_E_ARG;
    (void)hipSetDevice(G->e->device);
    const size_t n = (size_t)G->M * 3 * G->N;
    return G->e->precision == SP_F64 ? gneb_download<double>(G, G->x, chain, n) : gneb_download<float>(G, G->x, chain, n);
}

int sp_gneb_get_forces(sp_gneb* G, double* E, double* l, double* F) {
    if (!G) return SP_E_ARG;
    (void)hipSetDevice(G->e->device);
    if (hipStreamSynchronize(gneb_stream(G)) != hipSuccess) return gfail(G, SP_E_HIP, "synchronisation failed");
    if (E && hipMemcpy(E, G->E, G->M * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return gfail(G, SP_E_HIP, "download failed");
    if (l) {
        std::vector<double> s3(3 * (size_t)G->M);
        if (hipMemcpy(s3.data(), G->s3, s3.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            return gfail(G, SP_E_HIP, "download failed");
        for (int v = 0; v + 1 < G->M; ++v) l[v] = std::sqrt(s3[3 * v + 2]);
    }
    if (F) {
        const size_t n = (size_t)G->M * 3 * G->N;
        return G->e->precision == SP_F64 ? gneb_download<double>(G, G->Fp, F, n) : gneb_download<float>(G, G->Fp, F, n);
    }
    return SP_OK;
}

}  // extern "C"

// ================================================================= surrogate
#include "surrogate_host.inc"

// ====================================================================== FFT dipole
#include "fft_host.inc"

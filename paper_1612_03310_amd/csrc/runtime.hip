// Runtime of the MI355X path: device state, work tables, step scheduling,
// hipGraph replay, tile autotuning and the C ABI of include/mithra.h.
//
// A single simulation is a batch of one: every simulation of a batch lives in
// concatenated arenas and each kernel kind is one launch per step for all of
// them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mithra.h"
#include "mithra_internal.hpp"

namespace mithra {

// CODATA 2018
static const double C_LIGHT = 299792458.0;
static const double QE_C = 1.602176634e-19;
static const double ME_KG = 9.1093837015e-31;
static const double EPS0 = 8.8541878128e-12;
static const double MU0 = 1.0 / (EPS0 * C_LIGHT * C_LIGHT);
static const double PI = 3.14159265358979323846;

static thread_local std::string g_err;

// Scratch of the allocation-free read-back (mithra_get_field_noalloc): the six
// vertex-field components of NOALLOC_CELLS cells, or one field widened to
// double.  Each GPU the library runs on holds its own copy until the process
// ends; its address on a device comes from hipGetSymbolAddress, taken once
// per device when the first simulation is created there.
constexpr long long NOALLOC_CELLS = 1LL << 18;
static __device__ __align__(256) double scratch[6 * NOALLOC_CELLS];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];
static void *(*g_alloc)(size_t, void *) = nullptr;
static void (*g_free)(void *, void *) = nullptr;
static void *g_alloc_ctx = nullptr;

static mithra_status fail(mithra_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(MITHRA_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct HostSim {
    mithra_mesh mesh;
    mithra_undulator und;
    mithra_diag_cfg diag;
    mithra_seed seed{};  // amplitude 0: none
    mithra_seed optical{};  // optical undulator (wave towards -z); amplitude 0: static undulator
    mithra_beam beam{};     // its beam (type 0: plane wave)
    mithra_beam seed_beam{};        // the seed's beam (type 0: plane wave)
    double *seed_corr = nullptr;    // device: Gaussian-beam seed corrections
    bool has_bg = false;            // a static background charge is set
    void *bg = nullptr, *rho_bg = nullptr;  // device: background, rho + background
    double dt, dtb, A, gamma0, beta0, B0, ku;
    bool loaded = false;
    double q = 0.0, m = 0.0;
    // staged particles in split form (cell, offset, momentum, alive)
    std::vector<int> cell;    // 3 per particle
    std::vector<double> frac; // 3 per particle
    std::vector<double> mom;  // 3 per particle
    std::vector<unsigned char> alive;
    long long read_step = 0;
    // normalized frequencies of the plane spectrum and the step it (re)started
    int nfreq = 3;
    double fnu[MAXF] = {1.0, 2.0, 3.0};
    long long step0 = 0;
};

struct Batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // the re-binning (scan, scatter) runs on a second stream beside the deposit
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    mithra_precision prec = MITHRA_F64;
    size_t rs = 8;  // bytes per real
    int nsim = 0;
    std::vector<HostSim> hs;
    std::vector<SimDev> sd;
    long long total_cells = 0, total_keys = 0, total_particles = 0;
    long long total_spec = 0;  // doubles of the plane-spectrum arena
    Arena ar{};
    SimDev *d_sims = nullptr;
    // work tables
    int tile_x = 64, tile_y = 4, kz = 64;
    int fuse_x = 0;  // the stencil pass updates the x faces
    int4 *d_stencil = nullptr;
    int n_stencil = 0;
    BSeg *d_bseg = nullptr;
    int nbseg = 0;
    long long nb_total = 0;
    // second-order Mur: faces, edges, corners (one launch each, in order)
    BSeg *d_m2seg[3] = {nullptr, nullptr, nullptr};
    int nm2seg[3] = {0, 0, 0};
    long long nm2_total[3] = {0, 0, 0};
    int n_tiles = 0;
    // push and deposit: bricks of tiles dealt to the XCDs (shape from the tuner)
    int brick[3] = {32, 32, 2};  // whole tile layers by default (clipped to the grids)
    Brick *d_bricks = nullptr;
    int n_bricks = 0;
    int2 *d_plane = nullptr, *d_mesh = nullptr, *d_kin = nullptr;
    int n_plane = 0, n_mesh = 0, n_kin = 0;
    int *d_bsum = nullptr;
    int n_scan_blocks = 0;
    int4 *d_chunks = nullptr;  // per scan chunk: tiles it covers, lost bucket
    double *d_eb = nullptr;
    long long step = 0;
    bool committed = false;
    // graph replay
    bool use_graph = true;
    int graph_steps = 8;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // timing
    bool timing = false;
    double ms[NKINDS] = {0};
    long long calls[NKINDS] = {0};
    std::vector<int> ev_kind;
    std::vector<hipEvent_t> ev_a, ev_b;
    // memory
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *alloc_ctx = nullptr;
    // device blocks by lifetime: the batch, the particle arrays, the launch
    // tables, the diagnostic ring (re-laid when a ring capacity changes)
    struct Block {
        void *p;
        size_t bytes;
    };
    std::vector<Block> mem_fixed, mem_part, mem_tab, mem_ring, mem_spec;
    size_t bytes = 0;
};

// ---------------------------------------------------------------------------
// memory
// ---------------------------------------------------------------------------

static void *dev_alloc(Batch &b, size_t bytes, std::vector<Batch::Block> &owner)
{
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (b.alloc_fn) {
        p = b.alloc_fn(bytes, b.alloc_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) {
        owner.push_back({p, bytes});
        b.bytes += bytes;
    }
    return p;
}

static void dev_free_all(Batch &b, std::vector<Batch::Block> &owner)
{
    for (const Batch::Block &m : owner) {
        if (b.free_fn) b.free_fn(m.p, b.alloc_ctx);
        else (void)hipFree(m.p);
        b.bytes -= m.bytes;
    }
    owner.clear();
}

// some simulation has the optical undulator on (selects the push variant)
static int any_optical(const Batch &b)
{
    for (int s = 0; s < b.nsim; ++s)
        if (b.sd[s].opt_on) return 1;
    return 0;
}

static void drop_graph(Batch &b)
{
    if (b.gexec) (void)hipGraphExecDestroy(b.gexec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.gexec = nullptr;
    b.graph = nullptr;
}

static void destroy_batch(Batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->side) (void)hipStreamSynchronize(b->side);
    drop_graph(*b);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->side) (void)hipStreamDestroy(b->side);
    for (size_t i = 0; i < b->ev_a.size(); ++i) {
        (void)hipEventDestroy(b->ev_a[i]);
        (void)hipEventDestroy(b->ev_b[i]);
    }
    dev_free_all(*b, b->mem_tab);
    dev_free_all(*b, b->mem_part);
    dev_free_all(*b, b->mem_ring);
    dev_free_all(*b, b->mem_spec);
    dev_free_all(*b, b->mem_fixed);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

// ---------------------------------------------------------------------------
// validation and derived constants
// ---------------------------------------------------------------------------

static mithra_status validate(int s, const mithra_mesh &m, const mithra_undulator &u)
{
    for (int a = 0; a < 3; ++a) {
        if (m.n[a] < 8 || m.n[a] > (1 << 20))
            return fail(MITHRA_EINVAL, "sim %d: n[%d] = %d must be in [8, 2^20]", s, a, m.n[a]);
        if (!(m.d[a] > 0.0) || !std::isfinite(m.d[a]))
            return fail(MITHRA_EINVAL, "sim %d: d[%d] must be positive and finite", s, a);
        if (!std::isfinite(m.origin[a]))
            return fail(MITHRA_EINVAL, "sim %d: origin[%d] must be finite", s, a);
        if (m.bc[a] != MITHRA_BC_MUR1 && m.bc[a] != MITHRA_BC_PERIODIC &&
            m.bc[a] != MITHRA_BC_MUR2)
            return fail(MITHRA_EINVAL,
                        "sim %d: bc[%d] must be 0 (Mur-1), 1 (periodic) or 2 (Mur-2)", s, a);
    }
    {
        bool o1 = false, o2 = false;
        for (int a = 0; a < 3; ++a) {
            o1 |= m.bc[a] == MITHRA_BC_MUR1;
            o2 |= m.bc[a] == MITHRA_BC_MUR2;
        }
        if (o1 && o2)
            return fail(MITHRA_EINVAL, "sim %d: first- and second-order Mur axes cannot be mixed", s);
    }
    const double cells = (double)m.n[0] * m.n[1] * m.n[2];
    if (cells > 1.5e9) return fail(MITHRA_EINVAL, "sim %d: more than 1.5e9 grid points", s);
    if (!(m.courant > 0.0 && m.courant <= 1.0))
        return fail(MITHRA_EINVAL, "sim %d: courant = %g must be in (0, 1]", s, m.courant);
    if (m.substeps < 1) return fail(MITHRA_EINVAL, "sim %d: substeps must be >= 1", s);
    if (m.space_charge != 0 && m.space_charge != 1)
        return fail(MITHRA_EINVAL, "sim %d: space_charge must be 0 or 1", s);
    if (!(u.lambda_u > 0.0) || !std::isfinite(u.lambda_u))
        return fail(MITHRA_EINVAL, "sim %d: lambda_u must be positive", s);
    if (!(u.K >= 0.0) || !std::isfinite(u.K)) return fail(MITHRA_EINVAL, "sim %d: K must be >= 0", s);
    if (!std::isfinite(u.gamma_beam) || !std::isfinite(u.z_entrance))
        return fail(MITHRA_EINVAL, "sim %d: gamma_beam and z_entrance must be finite", s);
    if (!(u.gamma_beam / std::sqrt(1.0 + u.K * u.K / 2.0) > 1.0))
        return fail(MITHRA_EINVAL, "sim %d: gamma_beam / sqrt(1 + K^2/2) must exceed 1", s);
    if (!std::isfinite(u.length)) return fail(MITHRA_EINVAL, "sim %d: length must be finite", s);
    if (u.length > 0.0) {
        const double periods = u.length / u.lambda_u;
        if (std::fabs(periods - std::round(periods)) > 1e-9 * std::max(1.0, periods) ||
            std::round(periods) < 1.0)
            return fail(MITHRA_EINVAL,
                        "sim %d: length = %g m must be a whole number (>= 1) of periods of %g m",
                        s, u.length, u.lambda_u);
    }
    // stability: the right-hand side of the NSFD dispersion relation,
    // (c dt)^2 [(1 - 4 A sz)(sx/dx^2 + sy/dy^2) + sz/dz^2] with sx, sy, sz the
    // sin^2 terms in [0, 1], is multilinear, so its largest value sits at a
    // corner of the unit cube; it must not exceed 1.
    const double dx = m.d[0], dy = m.d[1], dz = m.d[2];
    const double A = m.nsfd_A < 0.0
                         ? 0.25 * (1.0 + 0.02 / ((dz / dx) * (dz / dx) + (dz / dy) * (dz / dy)))
                         : m.nsfd_A;
    const double cdt = m.courant * dz;
    double worst = 0.0;
    for (int c = 0; c < 8; ++c) {
        const double sx = c & 1, sy = (c >> 1) & 1, sz = (c >> 2) & 1;
        const double v = cdt * cdt * ((1.0 - 4.0 * A * sz) * (sx / (dx * dx) + sy / (dy * dy)) +
                                      sz / (dz * dz));
        worst = std::max(worst, v);
    }
    if (worst > 1.0 + 1e-12)
        return fail(MITHRA_EINVAL,
                    "sim %d: unstable mesh: the NSFD dispersion relation needs "
                    "(c dt)^2 [(1-4A sz)(sx/dx^2+sy/dy^2)+sz/dz^2] <= 1, worst corner %.6g "
                    "(A = %g; for c dt = dz use A >= 1/4 and (dz/dx)^2+(dz/dy)^2 < 1)",
                    s, worst, A);
    return MITHRA_OK;
}

static void derive(HostSim &h)
{
    const mithra_mesh &m = h.mesh;
    const double dx = m.d[0], dy = m.d[1], dz = m.d[2];
    h.dt = m.courant * dz / C_LIGHT;
    h.dtb = h.dt / m.substeps;
    h.A = m.nsfd_A < 0.0 ? 0.25 * (1.0 + 0.02 / ((dz / dx) * (dz / dx) + (dz / dy) * (dz / dy)))
                         : m.nsfd_A;
    h.gamma0 = h.und.gamma_beam / std::sqrt(1.0 + h.und.K * h.und.K / 2.0);
    h.beta0 = std::sqrt(1.0 - 1.0 / (h.gamma0 * h.gamma0));
    h.B0 = 2.0 * PI * ME_KG * C_LIGHT * h.und.K / (QE_C * h.und.lambda_u);
    h.ku = 2.0 * PI / h.und.lambda_u;
}

static void fill_seed(const HostSim &h, SimDev &S)
{
    S.seed_on = h.seed.amplitude != 0.0 ? 1 : 0;
    S.seed_sig = h.seed.signal;
    S.seed_a0 = h.seed.amplitude;
    S.seed_p[0] = h.seed.polarization[0];
    S.seed_p[1] = h.seed.polarization[1];
    S.seed_f = h.seed.frequency;
    S.seed_t0 = h.seed.t0;
    S.seed_tau = h.seed.tau > 0.0 ? h.seed.tau : 1.0;
    S.seed_cep = h.seed.cep;
    S.seed_zref = h.seed.z_ref;
    S.seed_beam = h.seed_beam.type;
    S.seed_zr[0] = h.seed_beam.rayleigh[0];
    S.seed_zr[1] = h.seed_beam.rayleigh[1];
    for (int a = 0; a < 3; ++a) S.seed_focus[a] = h.seed_beam.focus[a];
    S.seed_k = 2.0 * PI * h.seed.frequency / C_LIGHT;
    S.seed_corr = h.seed_corr;
}

// the simulation's step launches the Gaussian-beam seed kernel
static bool seed_beam_active(const SimDev &S)
{
    return S.seed_on && S.seed_beam == MITHRA_BEAM_GAUSSIAN && S.seed_corr != nullptr;
}

// which simulations launch the seed kernel (part of a captured step)
static std::vector<int> seed_beam_sims(const Batch &b)
{
    std::vector<int> v;
    for (int s = 0; s < b.nsim; ++s)
        if (seed_beam_active(b.sd[s])) v.push_back(s);
    return v;
}

static void fill_optical(const HostSim &h, SimDev &S)
{
    S.opt_on = h.optical.amplitude != 0.0 ? 1 : 0;
    S.opt_sig = h.optical.signal;
    S.opt_a = h.optical.amplitude;
    S.opt_p[0] = h.optical.polarization[0];
    S.opt_p[1] = h.optical.polarization[1];
    S.opt_f = h.optical.frequency;
    S.opt_t0 = h.optical.t0;
    S.opt_tau = h.optical.tau > 0.0 ? h.optical.tau : 1.0;
    S.opt_cep = h.optical.cep;
    S.opt_zref = h.optical.z_ref;
    S.opt_beam = h.beam.type;
    S.opt_zr[0] = h.beam.rayleigh[0];
    S.opt_zr[1] = h.beam.rayleigh[1];
    for (int a = 0; a < 3; ++a) S.opt_focus[a] = h.beam.focus[a];
    S.opt_k = 2.0 * PI * h.optical.frequency / C_LIGHT;
}

// fill the per-simulation constants (offsets are set by the layout)
// lab undulator position of the power plane at t = 0: z' = gamma0 (z_k - z_e),
// advancing at gamma0 beta0 c (z' = gamma0 (z - z_e + beta0 c t))
static double plate_position(const HostSim &h)
{
    return h.gamma0 * (h.mesh.origin[2] + h.diag.power_plane_k * h.mesh.d[2] - h.und.z_entrance);
}

static void fill_simdev(const HostSim &h, SimDev &S)
{
    const mithra_mesh &m = h.mesh;
    for (int a = 0; a < 3; ++a) {
        S.n[a] = m.n[a];
        S.bc[a] = m.bc[a] == MITHRA_BC_PERIODIC ? 1 : 0;
        S.nt[a] = (m.n[a] + TILE - 1) / TILE;
        S.d[a] = m.d[a];
        S.origin[a] = m.origin[a];
    }
    S.mur2 = (m.bc[0] == MITHRA_BC_MUR2 || m.bc[1] == MITHRA_BC_MUR2 || m.bc[2] == MITHRA_BC_MUR2)
                 ? 1
                 : 0;
    S.sc = m.space_charge;
    S.nsub = m.substeps;
    S.nkeys = S.nt[0] * S.nt[1] * S.nt[2] * TILE_CELLS;
    const double cdt = C_LIGHT * h.dt;
    const double nx2 = (cdt / m.d[0]) * (cdt / m.d[0]);
    const double ny2 = (cdt / m.d[1]) * (cdt / m.d[1]);
    const double nz2 = (cdt / m.d[2]) * (cdt / m.d[2]);
    S.A = h.A;
    S.a1 = 2.0 * (1.0 - (1.0 - 2.0 * h.A) * nx2 - (1.0 - 2.0 * h.A) * ny2 - nz2);
    S.ax = nx2;
    S.ay = ny2;
    S.az = nz2 - 2.0 * h.A * nx2 - 2.0 * h.A * ny2;
    S.srcA = cdt * cdt * MU0;
    S.srcPhi = cdt * cdt / EPS0;
    for (int a = 0; a < 3; ++a) {
        S.murb0[a] = (cdt - m.d[a]) / (cdt + m.d[a]);
        S.murb1[a] = 2.0 * m.d[a] / (cdt + m.d[a]);
        {
            // second-order face normal to a: transverse axes u < w
            const int u = a == 0 ? 1 : 0, w = a == 2 ? 1 : 2;
            const double h = m.d[a], ru = cdt / m.d[u], rw = cdt / m.d[w];
            S.murg[a][0] = (cdt - h) / (cdt + h);
            S.murg[a][1] = h * (2.0 - rw * rw - ru * ru) / (cdt + h);
            S.murg[a][2] = ru * ru * h / (2.0 * (cdt + h));
            S.murg[a][3] = rw * rw * h / (2.0 * (cdt + h));
        }
        S.inv_2d[a] = 0.5 / m.d[a];
        S.cdtb_d[a] = C_LIGHT * h.dtb / m.d[a];
    }
    S.inv_dt = 1.0 / h.dt;
    S.dt = h.dt;
    S.dtb = h.dtb;
    S.ku = h.ku;
    S.kz_cell = h.ku * h.gamma0 * m.d[2];
    S.phase_off = h.ku * h.gamma0 * (m.origin[2] - h.und.z_entrance);
    S.phase_rate = h.ku * h.gamma0 * h.beta0 * C_LIGHT;
    const double q = h.loaded ? h.q : -QE_C, mm = h.loaded ? h.m : ME_KG;
    S.kE = q * h.dtb / (2.0 * mm * C_LIGHT);
    S.kB = q * h.dtb / (2.0 * mm);
    S.EuK = S.kE * (-h.gamma0 * h.beta0 * C_LIGHT) * h.B0;
    S.BuyK = S.kB * h.gamma0 * h.B0;
    S.BuzK = S.kB * h.B0;
    const double dV = m.d[0] * m.d[1] * m.d[2];
    // deposit units per particle weight (the fixed-point scale is applied
    // per tile by the deposit)
    S.rho_unit = q / dV;
    for (int a = 0; a < 3; ++a) S.J_unit[a] = -q * m.d[a] / (dV * h.dt);
    S.dV = dV;
    fill_seed(h, S);
    fill_optical(h, S);
    S.mc2 = mm * C_LIGHT * C_LIGHT;
    S.dxdy_mu0 = m.d[0] * m.d[1] / MU0;
    S.eps0_half = 0.5 * EPS0;
    S.inv_2mu0 = 0.5 / MU0;
    S.kbunch = 2.0 * h.gamma0 * h.ku;
    S.omega1 = h.gamma0 * h.beta0 * C_LIGHT * h.ku;
    S.nfreq = h.nfreq;
    for (int f = 0; f < MAXF; ++f) S.fnu[f] = f < h.nfreq ? h.fnu[f] : 0.0;
    S.step0 = h.step0;
    S.lab_g = h.gamma0;
    S.lab_gb = h.gamma0 * h.beta0;
    S.zu0 = plate_position(h);
    S.zu_rate = h.gamma0 * h.beta0 * C_LIGHT;
    S.und_kL = h.und.length > 0.0 ? h.ku * h.und.length : 0.0;
    S.probe[0] = h.diag.probe[0];
    S.probe[1] = h.diag.probe[1];
    S.probe[2] = h.diag.probe[2];
    S.kp = h.diag.power_plane_k;
    S.mesh_every = h.diag.mesh_diag_every;
    S.ring_cap = h.diag.capacity;
    S.spec_on = h.diag.power_spectrum ? 1 : 0;
    S.n_extra = 0;
    for (int e = 0; e < 3; ++e)
        if (h.diag.extra_planes[e] >= 0) S.kp_extra[S.n_extra++] = h.diag.extra_planes[e];
    S.bg = h.has_bg ? h.bg : nullptr;
    S.rho_bg = h.has_bg ? h.rho_bg : nullptr;
}

// which simulations add a background charge before the potential update
static std::vector<int> background_sims(const Batch &b)
{
    std::vector<int> v;
    for (int s = 0; s < b.nsim; ++s)
        if (b.sd[s].rho_bg) v.push_back(s);
    return v;
}

static int tile_key_host(const SimDev &S, int ci, int cj, int ck)
{
    const int t = ((ck >> 3) * S.nt[1] + (cj >> 3)) * S.nt[0] + (ci >> 3);
    return t * TILE_CELLS + (((ck & 7) * TILE + (cj & 7)) * TILE + (ci & 7));
}

// ---------------------------------------------------------------------------
// work tables
// ---------------------------------------------------------------------------

template <typename T>
static mithra_status upload_table(Batch &b, const std::vector<T> &v, T **dst)
{
    *dst = (T *)dev_alloc(b, std::max<size_t>(1, v.size()) * sizeof(T), b.mem_tab);
    if (!*dst) return fail(MITHRA_ENOMEM, "device allocation of a work table failed");
    if (!v.empty())
        HIP_TRY(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice,
                               b.stream));
    return MITHRA_OK;
}

static void stencil_items(const Batch &b, int tx, int ty, int kz, std::vector<int4> &out)
{
    out.clear();
    for (int s = 0; s < b.nsim; ++s) {
        const SimDev &S = b.sd[s];
        const int bx = (S.n[0] + tx - 1) / tx, by = (S.n[1] + ty - 1) / ty,
                  bz = (S.n[2] + kz - 1) / kz;
        for (int z = 0; z < bz; ++z)
            for (int y = 0; y < by; ++y)
                for (int x = 0; x < bx; ++x) out.push_back(make_int4(s, x, y, z));
    }
}

// The deposit skips rewriting zeros into tiles whose sources are known to be
// zero; after any write from the host every tile is taken as non-zero.
static hipError_t mark_sources_dirty(Batch &b)
{
    const size_t tb = sizeof(int) * std::max(b.n_tiles, 1);
    hipError_t e = hipMemsetAsync(b.ar.jdirty, 1, tb, b.stream);
    for (int r = 0; r < 2 && e == hipSuccess; ++r) e = hipMemsetAsync(b.ar.rdirty[r], 1, tb, b.stream);
    return e;
}

// The stencil can update the x faces when every face column has its inward
// neighbour in the same wavefront row: the low face (x = 0) always does, the
// high face (x = ext - 1) unless it is the first lane of a wavefront.
static bool x_faces_fusable(const Batch &b, int tx)
{
    if (tx < 2) return false;
    for (int s = 0; s < b.nsim; ++s) {
        const SimDev &S = b.sd[s];
        if (S.bc[0]) continue;
        for (int c = 0; c < 4; ++c) {
            if (c == 3 && !S.sc) continue;
            const int ext = c == 0 ? S.n[0] - 1 : S.n[0];
            if ((ext - 1) % tx % 64 == 0) return false;
        }
    }
    return true;
}

// the bricks of every simulation's tile grid, in order (x fastest)
static void brick_table(const Batch &b, const int shape[3], std::vector<Brick> &out)
{
    out.clear();
    for (int s = 0; s < b.nsim; ++s) {
        const SimDev &S = b.sd[s];
        for (int z = 0; z < S.nt[2]; z += shape[2])
            for (int y = 0; y < S.nt[1]; y += shape[1])
                for (int x = 0; x < S.nt[0]; x += shape[0]) {
                    Brick br;
                    br.sim = s;
                    br.g0 = S.tile0 + (z * S.nt[1] + y) * S.nt[0] + x;
                    br.t0[0] = x;
                    br.t0[1] = y;
                    br.t0[2] = z;
                    for (int a = 0; a < 3; ++a) br.nt[a] = S.nt[a];
                    out.push_back(br);
                }
    }
}

static int4 brick_shape(const int shape[3])
{
    return make_int4(shape[0], shape[1], shape[2], shape[0] * shape[1] * shape[2]);
}

static mithra_status build_tables(Batch &b)
{
    (void)hipStreamSynchronize(b.stream);
    dev_free_all(b, b.mem_tab);
    b.d_eb = nullptr;
    drop_graph(b);
    mithra_status st;
    // stencil
    std::vector<int4> items;
    stencil_items(b, b.tile_x, b.tile_y, b.kz, items);
    b.n_stencil = (int)items.size();
    if ((st = upload_table(b, items, &b.d_stencil))) return st;
    // boundary segments (Mur axes only; the x faces go with the stencil when
    // it can take them)
    b.fuse_x = x_faces_fusable(b, b.tile_x) ? 1 : 0;
    std::vector<BSeg> segs;
    long long start = 0;
    for (int s = 0; s < b.nsim; ++s) {
        const SimDev &S = b.sd[s];
        if (S.mur2) continue;
        for (int c = 0; c < 4; ++c) {
            if (c == 3 && !S.sc) continue;
            int ext[3], ni[3];
            for (int a = 0; a < 3; ++a) {
                ext[a] = (c == a && !S.bc[a]) ? S.n[a] - 1 : S.n[a];
                ni[a] = S.bc[a] ? ext[a] : ext[a] - 2;
            }
            const long long cnt[3] = {2LL * ni[1] * ni[2], 2LL * ext[0] * ni[2],
                                      2LL * ext[0] * ext[1]};
            for (int g = 2; g >= 0; --g) {
                if (S.bc[g] || (g == 0 && b.fuse_x)) continue;
                BSeg sg;
                sg.sim = s;
                sg.comp = c;
                sg.group = g;
                sg.pad = 0;
                sg.start = start;
                sg.count = cnt[g];
                start += cnt[g];
                segs.push_back(sg);
            }
        }
    }
    b.nbseg = (int)segs.size();
    b.nb_total = start;
    if ((st = upload_table(b, segs, &b.d_bseg))) return st;
    // second-order Mur: faces without their edges (group = face axis), edges
    // without their corners (group 3 + edge axis), corners (group 6)
    for (int stage = 0; stage < 3; ++stage) {
        std::vector<BSeg> m2;
        long long st2 = 0;
        for (int s = 0; s < b.nsim; ++s) {
            const SimDev &S = b.sd[s];
            if (!S.mur2) continue;
            for (int c = 0; c < 4; ++c) {
                if (c == 3 && !S.sc) continue;
                int ext[3], ni[3];
                for (int a = 0; a < 3; ++a) {
                    ext[a] = (c == a && !S.bc[a]) ? S.n[a] - 1 : S.n[a];
                    ni[a] = S.bc[a] ? ext[a] : ext[a] - 2;
                }
                auto add = [&](int group, long long count) {
                    BSeg sg;
                    sg.sim = s;
                    sg.comp = c;
                    sg.group = group;
                    sg.pad = 0;
                    sg.start = st2;
                    sg.count = count;
                    st2 += count;
                    m2.push_back(sg);
                };
                for (int a = 0; a < 3; ++a) {
                    const int u = a == 0 ? 1 : 0, w = a == 2 ? 1 : 2;
                    if (stage == 0 && !S.bc[a] && !(a == 0 && b.fuse_x)) add(a, 2LL * ni[u] * ni[w]);
                    if (stage == 1 && !S.bc[u] && !S.bc[w]) add(3 + a, 4LL * ni[a]);
                }
                if (stage == 2 && !S.bc[0] && !S.bc[1] && !S.bc[2]) add(6, 8);
            }
        }
        b.nm2seg[stage] = (int)m2.size();
        b.nm2_total[stage] = st2;
        if ((st = upload_table(b, m2, &b.d_m2seg[stage]))) return st;
    }
    // tiles
    std::vector<int2> plane, mesh, kin;
    int slot = 0, ntiles = 0;
    for (int s = 0; s < b.nsim; ++s) {
        SimDev &S = b.sd[s];
        S.tile0 = ntiles;
        ntiles += S.nt[0] * S.nt[1] * S.nt[2];
        const long long ncell = (long long)S.n[0] * S.n[1] * S.n[2];
        S.nb_plane = (S.n[0] * S.n[1] + BLOCK - 1) / BLOCK;
        S.nb_mesh = S.mesh_every > 0
                        ? (int)((ncell + BLOCK * MESH_DIAG_PER_THREAD - 1) / (BLOCK * MESH_DIAG_PER_THREAD))
                        : 0;
        S.nb_kin = S.mesh_every > 0 ? (int)((S.np + BLOCK * KIN_PER_THREAD - 1) / (BLOCK * KIN_PER_THREAD))
                                    : 0;
        S.part_plane0 = slot;
        slot += PLANE_STRIDE * S.nb_plane;
        S.part_extra0 = slot;
        slot += S.n_extra * S.nb_plane;
        S.part_mesh0 = slot;
        slot += 4 * S.nb_mesh;
        S.part_kin0 = slot;
        slot += KIN_TERMS * S.nb_kin;
        // plate p (0 the main one) block i is item y = p * nb_plane + i
        for (int i = 0; i < (1 + S.n_extra) * S.nb_plane; ++i) plane.push_back(make_int2(s, i));
        for (int i = 0; i < S.nb_mesh; ++i) mesh.push_back(make_int2(s, i));
        for (int i = 0; i < S.nb_kin; ++i) kin.push_back(make_int2(s, i));
    }
    b.n_tiles = ntiles;
    for (int a = 0; a < 3; ++a) {
        int mt = 1;
        for (int s = 0; s < b.nsim; ++s) mt = std::max(mt, b.sd[s].nt[a]);
        b.brick[a] = std::max(1, std::min(b.brick[a], mt));
    }
    std::vector<Brick> bricks;
    brick_table(b, b.brick, bricks);
    b.n_bricks = (int)bricks.size();
    b.n_plane = (int)plane.size();
    b.n_mesh = (int)mesh.size();
    b.n_kin = (int)kin.size();
    if ((st = upload_table(b, bricks, &b.d_bricks))) return st;
    if ((st = upload_table(b, plane, &b.d_plane))) return st;
    if ((st = upload_table(b, mesh, &b.d_mesh))) return st;
    if ((st = upload_table(b, kin, &b.d_kin))) return st;
    b.ar.partial = (double *)dev_alloc(b, sizeof(double) * std::max(slot, 1), b.mem_tab);
    b.n_scan_blocks = (int)((b.total_keys + SCAN_CHUNK - 1) / SCAN_CHUNK);
    b.d_bsum = (int *)dev_alloc(b, sizeof(int) * std::max(b.n_scan_blocks, 1), b.mem_tab);
    // per chunk of keys: the first and last global tile it covers and whether
    // it holds a lost bucket (the scan skips chunks whose tiles are all
    // unoccupied and that hold none); the host table lives until the stream
    // is synchronized below
    std::vector<int4> chunks((size_t)std::max(b.n_scan_blocks, 1), make_int4(INT_MAX, -1, 0, 0));
    {
        for (int s = 0; s < b.nsim; ++s) {
            const SimDev &S = b.sd[s];
            const int nt = S.nt[0] * S.nt[1] * S.nt[2];
            for (int t = 0; t < nt; ++t) {
                const long long k = S.key0 + (long long)t * TILE_CELLS;
                const long long c0 = k / SCAN_CHUNK, c1 = (k + TILE_CELLS - 1) / SCAN_CHUNK;
                for (long long c = c0; c <= c1; ++c) {
                    chunks[c].x = std::min(chunks[c].x, S.tile0 + t);
                    chunks[c].y = std::max(chunks[c].y, S.tile0 + t);
                }
            }
            chunks[(S.key0 + S.nkeys) / SCAN_CHUNK].z = 1;
        }
        for (int4 &c : chunks)
            if (c.x > c.y) c.x = 0, c.y = -1;  // no tile
        if ((st = upload_table(b, chunks, &b.d_chunks))) return st;
    }
    const size_t tb = sizeof(int) * std::max(b.n_tiles, 1);
    b.ar.tact = (int *)dev_alloc(b, tb, b.mem_tab);
    b.ar.jdirty = (int *)dev_alloc(b, tb, b.mem_tab);
    for (int r = 0; r < 2; ++r) b.ar.pocc[r] = (int *)dev_alloc(b, tb, b.mem_tab);
    for (int r = 0; r < 2; ++r) b.ar.rdirty[r] = (int *)dev_alloc(b, tb, b.mem_tab);
    if (!b.ar.partial || !b.d_bsum || !b.ar.tact || !b.ar.jdirty || !b.ar.rdirty[0] ||
        !b.ar.rdirty[1] || !b.ar.pocc[0] || !b.ar.pocc[1])
        return fail(MITHRA_ENOMEM, "device allocation failed");
    HIP_TRY(hipMemsetAsync(b.ar.partial, 0, sizeof(double) * std::max(slot, 1), b.stream));
    HIP_TRY(hipMemsetAsync(b.ar.tact, 0, tb, b.stream));
    // every tile may hold particles until a push says otherwise
    for (int r = 0; r < 2; ++r) HIP_TRY(hipMemsetAsync(b.ar.pocc[r], 1, tb, b.stream));
    HIP_TRY(mark_sources_dirty(b));
    HIP_TRY(hipMemcpyAsync(b.d_sims, b.sd.data(), sizeof(SimDev) * b.nsim, hipMemcpyHostToDevice,
                           b.stream));
    HIP_TRY(hipStreamSynchronize(b.stream));
    return MITHRA_OK;
}

// ---------------------------------------------------------------------------
// creation
// ---------------------------------------------------------------------------

// Lay out the diagnostic ring, the per-row spectrum arena and (spec) the
// plane-spectrum arena from each simulation's ring capacity and number of
// frequencies; the old arenas are freed once the new ones are in place.
// Only before the first step: no rows exist yet and the spectrum is zero.
static mithra_status relay_diag_arenas(Batch &b, bool spec)
{
    long long ring = 0, srow = 0, plate = 0;
    for (int i = 0; i < b.nsim; ++i) {
        const HostSim &h = b.hs[i];
        ring += h.diag.capacity;
        srow += (long long)h.diag.capacity * 2 * h.nfreq;
        plate += (long long)h.mesh.n[0] * h.mesh.n[1] * SPEC_PER_FREQ * h.nfreq;
    }
    std::vector<Batch::Block> fr, fs;
    double *nr = (double *)dev_alloc(b, sizeof(double) * NDIAG * ring, fr);
    double *nsr = nr ? (double *)dev_alloc(b, sizeof(double) * srow, fr) : nullptr;
    double *nsp = nullptr;
    if (nsr && spec) nsp = (double *)dev_alloc(b, sizeof(double) * plate, fs);
    hipError_t e = hipSuccess;
    if (nsr && (!spec || nsp)) {
        e = hipMemset(nr, 0, sizeof(double) * NDIAG * ring);
        if (e == hipSuccess) e = hipMemset(nsr, 0, sizeof(double) * srow);
        if (e == hipSuccess && spec) e = hipMemset(nsp, 0, sizeof(double) * plate);
    }
    if (!nsr || (spec && !nsp) || e != hipSuccess) {
        dev_free_all(b, fr);
        dev_free_all(b, fs);
        return e != hipSuccess ? fail(MITHRA_EDEVICE, "clearing the diagnostic arenas failed")
                               : fail(MITHRA_ENOMEM, "device allocation of the diagnostic arenas failed");
    }
    drop_graph(b);
    dev_free_all(b, b.mem_ring);
    b.mem_ring = fr;
    b.ar.ring = nr;
    b.ar.srow = nsr;
    if (spec) {
        dev_free_all(b, b.mem_spec);
        b.mem_spec = fs;
        b.ar.spec = nsp;
        b.total_spec = plate;
    }
    ring = srow = plate = 0;
    for (int i = 0; i < b.nsim; ++i) {
        const HostSim &h = b.hs[i];
        SimDev &S = b.sd[i];
        S.ring0 = ring;
        S.ring_cap = h.diag.capacity;
        S.srow0 = srow;
        ring += h.diag.capacity;
        srow += (long long)h.diag.capacity * 2 * h.nfreq;
        if (spec) {
            S.spec0 = plate;
            plate += (long long)h.mesh.n[0] * h.mesh.n[1] * SPEC_PER_FREQ * h.nfreq;
        }
    }
    return MITHRA_OK;
}

static mithra_status create_batch(int nsim, const mithra_mesh *meshes, const mithra_undulator *unds,
                                  mithra_precision prec, void *stream, Batch **out)
{
    if (!out) return fail(MITHRA_EINVAL, "out is NULL");
    *out = nullptr;
    if (nsim < 1 || !meshes || !unds) return fail(MITHRA_EINVAL, "need nsim >= 1 meshes and undulators");
    if (prec != MITHRA_F64 && prec != MITHRA_F32_SPLIT)
        return fail(MITHRA_EINVAL, "precision must be MITHRA_F64 or MITHRA_F32_SPLIT");
    for (int s = 0; s < nsim; ++s) {
        mithra_status st = validate(s, meshes[s], unds[s]);
        if (st) return st;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(MITHRA_EDEVICE, "device %d is %s; this library is built for gfx950 only", dev,
                    prop.gcnArchName);

    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(MITHRA_EDEVICE, "device index %d beyond the %d the library supports", dev,
                    MAX_DEVICES);
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *ptr = nullptr;
            hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(MITHRA_EDEVICE, "address of the read-back scratch on device %d: %s",
                            dev, hipGetErrorString(e));
            g_scratch_ptr[dev] = ptr;
        }
    }
    Batch *b = new Batch();
    b->device = dev;
    b->prec = prec;
    b->rs = prec == MITHRA_F64 ? 8 : 4;
    b->nsim = nsim;
    b->alloc_fn = g_alloc;
    b->free_fn = g_free;
    b->alloc_ctx = g_alloc_ctx;
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return fail(MITHRA_EDEVICE, "hipStreamCreateWithFlags failed");
        }
        b->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess) {
        destroy_batch(b);
        return fail(MITHRA_EDEVICE, "creating the second stream or its events failed");
    }
    b->hs.resize(nsim);
    b->sd.resize(nsim);
    long long cells = 0, keys = 0;
    for (int s = 0; s < nsim; ++s) {
        HostSim &h = b->hs[s];
        h.mesh = meshes[s];
        h.und = unds[s];
        h.diag.probe[0] = h.mesh.n[0] / 2;
        h.diag.probe[1] = h.mesh.n[1] / 2;
        h.diag.probe[2] = h.mesh.n[2] / 2;
        h.diag.power_plane_k = h.mesh.n[2] / 2;
        h.diag.mesh_diag_every = 1;
        h.diag.capacity = 4096;
        for (int e = 0; e < 3; ++e) h.diag.extra_planes[e] = -1;
        derive(h);
        SimDev &S = b->sd[s];
        std::memset(&S, 0, sizeof S);
        fill_simdev(h, S);
        S.cell0 = cells;
        S.key0 = keys;
        cells += (long long)S.n[0] * S.n[1] * S.n[2];
        keys += (long long)S.nkeys + 1;
    }
    if (keys >= (1LL << 31) - 1) {
        destroy_batch(b);
        return fail(MITHRA_EINVAL, "too many cells for 32-bit bin keys (%lld)", keys);
    }
    b->total_cells = cells;
    b->total_keys = keys;
    // default stencil shape, clamped to the meshes
    int maxn[3] = {0, 0, 0};
    for (int s = 0; s < nsim; ++s)
        for (int a = 0; a < 3; ++a) maxn[a] = std::max(maxn[a], b->sd[s].n[a]);
    if (maxn[0] <= 32) {
        b->tile_x = 32;
        b->tile_y = 8;
    }
    b->kz = std::min(64, maxn[2]);

    auto A = [&](size_t bytes) { return dev_alloc(*b, bytes, b->mem_fixed); };
    bool ok = true;
    const size_t mb = (size_t)cells * b->rs;
    for (int l = 0; l < 3; ++l)
        for (int c = 0; c < 4; ++c) ok &= (b->ar.pot[l][c] = A(mb)) != nullptr;
    for (int c = 0; c < 3; ++c) ok &= (b->ar.J[c] = A(mb)) != nullptr;
    for (int r = 0; r < 2; ++r) ok &= (b->ar.rho[r] = A(mb)) != nullptr;
    ok &= (b->ar.counts = (int *)A(sizeof(int) * keys)) != nullptr;
    for (int r = 0; r < 2; ++r) ok &= (b->ar.offs[r] = (int *)A(sizeof(int) * (keys + 1))) != nullptr;
    ok &= (b->ar.flags = (int *)A(sizeof(int) * nsim)) != nullptr;
    ok &= (b->ar.d_step = (long long *)A(sizeof(long long))) != nullptr;
    ok &= (b->ar.fin_ctr = (int *)A(sizeof(int))) != nullptr;
    ok &= (b->d_sims = (SimDev *)A(sizeof(SimDev) * nsim)) != nullptr;
    if (!ok) {
        destroy_batch(b);
        return fail(MITHRA_ENOMEM, "device allocation of %.3f GB failed",
                    (double)(15 * mb + 12 * keys) / 1e9);
    }
    hipError_t e = hipSuccess;
    for (int l = 0; l < 3 && e == hipSuccess; ++l)
        for (int c = 0; c < 4 && e == hipSuccess; ++c) e = hipMemsetAsync(b->ar.pot[l][c], 0, mb, b->stream);
    for (int c = 0; c < 3 && e == hipSuccess; ++c) e = hipMemsetAsync(b->ar.J[c], 0, mb, b->stream);
    for (int r = 0; r < 2 && e == hipSuccess; ++r) e = hipMemsetAsync(b->ar.rho[r], 0, mb, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->ar.counts, 0, sizeof(int) * keys, b->stream);
    for (int r = 0; r < 2 && e == hipSuccess; ++r)
        e = hipMemsetAsync(b->ar.offs[r], 0, sizeof(int) * (keys + 1), b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->ar.flags, 0, sizeof(int) * nsim, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->ar.d_step, 0, sizeof(long long), b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->ar.fin_ctr, 0, sizeof(int), b->stream);
    if (e != hipSuccess) {
        destroy_batch(b);
        return fail(MITHRA_EDEVICE, "clearing device memory failed: %s", hipGetErrorString(e));
    }
    mithra_status st = relay_diag_arenas(*b, true);
    if (!st) st = build_tables(*b);
    if (st) {
        destroy_batch(b);
        return st;
    }
    *out = b;
    return MITHRA_OK;
}

// ---------------------------------------------------------------------------
// particles
// ---------------------------------------------------------------------------

// Bucket offsets and particle indices are 32-bit; the margin keeps the index
// arithmetic of a block running past the last particle inside int range.
constexpr long long MAX_PARTICLES = (1LL << 31) - (1LL << 20);

static mithra_status stage_particles(HostSim &h, int s, int64_t np, const double *pos,
                                     const double *u, double q, double m)
{
    if (np < 0) return fail(MITHRA_EINVAL, "sim %d: np < 0", s);
    if (np > 0 && (!pos || !u)) return fail(MITHRA_EINVAL, "sim %d: pos and u must not be NULL", s);
    if (np > MAX_PARTICLES)
        return fail(MITHRA_EINVAL, "sim %d: %lld particles, at most %lld", s, (long long)np,
                    MAX_PARTICLES);
    if (!std::isfinite(q) || !(m > 0.0) || !std::isfinite(m))
        return fail(MITHRA_EINVAL, "sim %d: q must be finite and m positive", s);
    h.cell.assign(3 * np, 0);
    h.frac.assign(3 * np, 0.0);
    h.mom.assign(3 * np, 0.0);
    h.alive.assign(np, 1);
    for (int64_t p = 0; p < np; ++p) {
        for (int a = 0; a < 3; ++a) {
            const double x = pos[3 * p + a], v = u[3 * p + a];
            if (!std::isfinite(x) || !std::isfinite(v))
                return fail(MITHRA_EINVAL, "sim %d: particle %lld has a non-finite coordinate", s,
                            (long long)p);
            const double xi = (x - h.mesh.origin[a]) / h.mesh.d[a];
            const double fl = std::floor(xi);
            const bool in = fl >= 2.0 && fl <= h.mesh.n[a] - 3.0;
            if (!in) h.alive[p] = 0;
            h.cell[3 * p + a] = in ? (int)fl : 0;
            double f = xi - fl;
            if (f >= 1.0) f = std::nextafter(1.0, 0.0);
            h.frac[3 * p + a] = f;
            h.mom[3 * p + a] = v;
        }
    }
    h.q = q;
    h.m = m;
    h.loaded = true;
    return MITHRA_OK;
}

template <typename R>
static void fill_particle_arrays(Batch &b, std::vector<int> &key, std::vector<R> off[3],
                                 std::vector<R> uu[3], std::vector<int> &id,
                                 std::vector<int> &offs)
{
    const long long N = b.total_particles;
    key.assign(N, 0);
    id.assign(N, 0);
    for (int a = 0; a < 3; ++a) {
        off[a].assign(N, 0);
        uu[a].assign(N, 0);
    }
    // counting sort of all particles by global key
    std::vector<int> cnt(b.total_keys + 1, 0);
    std::vector<int> gkey(N);
    long long p0 = 0;
    for (int s = 0; s < b.nsim; ++s) {
        const HostSim &h = b.hs[s];
        const SimDev &S = b.sd[s];
        const long long np = (long long)h.alive.size();
        for (long long p = 0; p < np; ++p) {
            int k = S.nkeys;
            if (h.alive[p]) k = tile_key_host(S, h.cell[3 * p], h.cell[3 * p + 1], h.cell[3 * p + 2]);
            gkey[p0 + p] = (int)S.key0 + k;
            cnt[(int)S.key0 + k]++;
        }
        p0 += np;
    }
    offs.assign(b.total_keys + 1, 0);
    long long run = 0;
    for (long long g = 0; g < b.total_keys; ++g) {
        offs[g] = (int)run;
        run += cnt[g];
    }
    offs[b.total_keys] = (int)run;
    std::vector<int> cur(offs.begin(), offs.end() - 1);
    p0 = 0;
    for (int s = 0; s < b.nsim; ++s) {
        const HostSim &h = b.hs[s];
        const long long np = (long long)h.alive.size();
        for (long long p = 0; p < np; ++p) {
            const int g = gkey[p0 + p];
            const int dst = cur[g]++;
            key[dst] = g;
            id[dst] = (int)p;
            for (int a = 0; a < 3; ++a) {
                off[a][dst] = (R)h.frac[3 * p + a];
                // a float offset can round up to 1.0: keep it inside the cell
                if (!(off[a][dst] < (R)1)) off[a][dst] = std::nextafter((R)1, (R)0);
                uu[a][dst] = (R)h.mom[3 * p + a];
            }
        }
        p0 += np;
    }
}

template <typename R>
static mithra_status commit_impl(Batch &b)
{
    HIP_TRY(hipStreamSynchronize(b.stream));
    drop_graph(b);
    dev_free_all(b, b.mem_part);
    long long N = 0;
    for (int s = 0; s < b.nsim; ++s) N += (long long)b.hs[s].alive.size();
    if (N > MAX_PARTICLES)
        return fail(MITHRA_EINVAL, "%lld particles in the batch, at most %lld", N, MAX_PARTICLES);
    N = 0;
    for (int s = 0; s < b.nsim; ++s) {
        SimDev &S = b.sd[s];
        S.part0 = N;
        S.np = (int)b.hs[s].alive.size();
        N += S.np;
        const long long keep0 = S.cell0, keep1 = S.key0, keep2 = S.ring0, keep3 = S.part0,
                        keep4 = S.spec0, keep5 = S.srow0;
        const int np = S.np;
        // the plane spectrum restarts with the committed state
        b.hs[s].step0 = b.step;
        fill_simdev(b.hs[s], S);
        S.cell0 = keep0;
        S.key0 = keep1;
        S.ring0 = keep2;
        S.part0 = keep3;
        S.spec0 = keep4;
        S.srow0 = keep5;
        S.np = np;
    }
    b.total_particles = N;
    auto A = [&](size_t bytes) { return dev_alloc(b, bytes, b.mem_part); };
    bool ok = true;
    const size_t nr = (size_t)std::max(N, 1LL) * sizeof(R), ni = (size_t)std::max(N, 1LL) * sizeof(int);
    for (int r = 0; r < 2; ++r) {
        ok &= (b.ar.key[r] = (int *)A(ni)) != nullptr;
        ok &= (b.ar.id[r] = (int *)A(ni)) != nullptr;
        for (int a = 0; a < 3; ++a) {
            ok &= (b.ar.off[r][a] = A(nr)) != nullptr;
            ok &= (b.ar.u[r][a] = A(nr)) != nullptr;
        }
    }
    ok &= (b.ar.okey = (int *)A(ni)) != nullptr;
    for (int a = 0; a < 3; ++a) ok &= (b.ar.ooff[a] = A(nr)) != nullptr;
    ok &= (b.ar.ke = (double *)A(sizeof(double) * std::max(N, 1LL))) != nullptr;
    ok &= (b.ar.zr = (double *)A(sizeof(double) * std::max(N, 1LL))) != nullptr;
    if (!ok) return fail(MITHRA_ENOMEM, "device allocation for %lld particles failed", N);

    std::vector<int> key, id, offs;
    std::vector<R> off[3], uu[3];
    fill_particle_arrays<R>(b, key, off, uu, id, offs);
    const int par = (int)(b.step & 1);
    hipStream_t st = b.stream;
    if (N > 0) {
        HIP_TRY(hipMemcpyAsync(b.ar.key[par], key.data(), ni, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(b.ar.id[par], id.data(), ni, hipMemcpyHostToDevice, st));
        for (int a = 0; a < 3; ++a) {
            HIP_TRY(hipMemcpyAsync(b.ar.off[par][a], off[a].data(), nr, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(b.ar.u[par][a], uu[a].data(), nr, hipMemcpyHostToDevice, st));
        }
    }
    HIP_TRY(hipMemcpyAsync(b.ar.offs[par], offs.data(), sizeof(int) * (b.total_keys + 1),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(b.ar.counts, 0, sizeof(int) * b.total_keys, st));
    HIP_TRY(hipMemsetAsync(b.ar.ke, 0, sizeof(double) * std::max(N, 1LL), st));
    // the plane spectrum starts with the committed state
    HIP_TRY(hipMemsetAsync(b.ar.spec, 0, sizeof(double) * b.total_spec, st));
    // all-ones bytes are a NaN: no position until a live particle's first
    // diagnostic push, and none ever for a particle lost at loading
    HIP_TRY(hipMemsetAsync(b.ar.zr, 0xff, sizeof(double) * std::max(N, 1LL), st));
    HIP_TRY(hipMemsetAsync(b.ar.flags, 0, sizeof(int) * b.nsim, st));
    // the step counter on the device must match the host mirror
    HIP_TRY(hipMemcpyAsync(b.ar.d_step, &b.step, sizeof(long long), hipMemcpyHostToDevice, st));
    mithra_status s2 = build_tables(b);
    if (s2) return s2;
    // rho^{s+1/2} from the loaded positions; J^s = 0 (start = end position)
    launch_deposit<R>(st, b.d_sims, b.d_bricks, b.n_bricks, brick_shape(b.brick), b.ar, 1);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    b.committed = true;
    return MITHRA_OK;
}

static mithra_status commit(Batch &b)
{
    for (int s = 0; s < b.nsim; ++s)
        if (!b.hs[s].loaded) return fail(MITHRA_ESTATE, "sim %d has no particles loaded", s);
    return b.prec == MITHRA_F64 ? commit_impl<double>(b) : commit_impl<float>(b);
}

// ---------------------------------------------------------------------------
// stepping
// ---------------------------------------------------------------------------

static hipEvent_t new_event()
{
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

template <typename R>
static void enqueue_step(Batch &b, bool timed)
{
    hipStream_t st = b.stream;
    auto mark = [&](int kind, bool begin) {
        if (!timed) return;
        if (begin) {
            b.ev_kind.push_back(kind);
            b.ev_a.push_back(new_event());
            b.ev_b.push_back(new_event());
            (void)hipEventRecord(b.ev_a.back(), st);
        } else {
            (void)hipEventRecord(b.ev_b.back(), st);
        }
    };
    mark(K_STENCIL, true);
    for (int s : seed_beam_sims(b))
        launch_seed_beam(st, b.d_sims, s, b.sd[s].n[0] * b.sd[s].n[1], b.ar.d_step);
    for (int s : background_sims(b))
        launch_background<R>(st, b.d_sims, s, (long long)b.sd[s].n[0] * b.sd[s].n[1] * b.sd[s].n[2],
                             b.ar);
    launch_stencil<R>(st, b.d_sims, b.d_stencil, b.n_stencil, b.ar, b.tile_x, b.tile_y, b.kz,
                      b.fuse_x);
    mark(K_STENCIL, false);
    mark(K_BOUNDARY, true);
    launch_boundary<R>(st, b.d_sims, b.d_bseg, b.nbseg, b.nb_total, b.ar);
    for (int stage = 0; stage < 3; ++stage)
        launch_mur2<R>(st, b.d_sims, b.d_m2seg[stage], b.nm2seg[stage], b.nm2_total[stage], b.ar);
    mark(K_BOUNDARY, false);
    mark(K_PUSH, true);
    launch_push<R>(st, b.d_sims, b.d_bricks, b.n_bricks, brick_shape(b.brick), b.ar,
                   any_optical(b));
    mark(K_PUSH, false);
    if (timed) {
        // one stream, so that each kind's events bracket that kind alone
        mark(K_DEPOSIT, true);
        launch_deposit<R>(st, b.d_sims, b.d_bricks, b.n_bricks, brick_shape(b.brick), b.ar, 0);
        mark(K_DEPOSIT, false);
        mark(K_SCAN, true);
        launch_scan(st, b.ar, b.total_keys, b.d_bsum, b.n_scan_blocks, b.d_chunks);
        mark(K_SCAN, false);
        mark(K_SCATTER, true);
        launch_scatter<R>(st, b.ar, b.total_particles);
        mark(K_SCATTER, false);
    } else {
        // The deposit reads the particle buffer of this step, its bucket
        // starts and start records; the scan writes the other bucket starts
        // and the scatter the other particle buffer.  Nothing is shared, so
        // the re-binning runs on the second stream while the deposit runs.
        (void)hipEventRecord(b.ev_fork, st);
        (void)hipStreamWaitEvent(b.side, b.ev_fork, 0);
        launch_scan(b.side, b.ar, b.total_keys, b.d_bsum, b.n_scan_blocks, b.d_chunks);
        launch_scatter<R>(b.side, b.ar, b.total_particles);
        (void)hipEventRecord(b.ev_join, b.side);
        launch_deposit<R>(st, b.d_sims, b.d_bricks, b.n_bricks, brick_shape(b.brick), b.ar, 0);
        (void)hipStreamWaitEvent(st, b.ev_join, 0);
    }
    mark(K_DIAG, true);
    launch_diag<R>(st, b.d_sims, b.nsim, b.d_plane, b.n_plane, b.d_mesh, b.n_mesh, b.d_kin,
                   b.n_kin, b.ar);
    mark(K_DIAG, false);
}

template <typename R>
static mithra_status run_impl(Batch &b, int64_t nsteps)
{
    if (b.timing || !b.use_graph) {
        for (int64_t i = 0; i < nsteps; ++i) enqueue_step<R>(b, b.timing);
        HIP_TRY(hipGetLastError());
        b.step += nsteps;
        return MITHRA_OK;
    }
    // The step graph is captured and instantiated on the first run after
    // any change of the launch tables, whatever its length, so that the
    // one-off cost of building it falls on that run and not on a later,
    // longer one; runs replay it G steps at a time and enqueue the rest
    // directly.
    const int G = b.graph_steps;
    if (!b.gexec) {
        HIP_TRY(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < G; ++i) enqueue_step<R>(b, false);
        hipError_t e = hipStreamEndCapture(b.stream, &b.graph);
        if (e != hipSuccess) {
            b.graph = nullptr;
            return fail(MITHRA_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        }
        e = hipGraphInstantiate(&b.gexec, b.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return fail(MITHRA_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
        }
    }
    int64_t done = 0;
    while (nsteps - done >= G) {
        HIP_TRY(hipGraphLaunch(b.gexec, b.stream));
        done += G;
    }
    for (; done < nsteps; ++done) enqueue_step<R>(b, false);
    HIP_TRY(hipGetLastError());
    b.step += nsteps;
    return MITHRA_OK;
}

static mithra_status run(Batch &b, int64_t nsteps)
{
    if (nsteps < 0) return fail(MITHRA_EINVAL, "nsteps < 0");
    HIP_TRY(hipSetDevice(b.device));
    if (!b.committed) {
        mithra_status st = commit(b);
        if (st) return st;
    }
    if (nsteps == 0) return MITHRA_OK;
    return b.prec == MITHRA_F64 ? run_impl<double>(b, nsteps) : run_impl<float>(b, nsteps);
}

// wait for the stream and fold the timing events into the totals
static mithra_status sync_stream(Batch &b)
{
    HIP_TRY(hipSetDevice(b.device));
    HIP_TRY(hipStreamSynchronize(b.stream));
    for (size_t i = 0; i < b.ev_kind.size(); ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, b.ev_a[i], b.ev_b[i]) == hipSuccess) {
            b.ms[b.ev_kind[i]] += ms;
            b.calls[b.ev_kind[i]] += 1;
        }
        (void)hipEventDestroy(b.ev_a[i]);
        (void)hipEventDestroy(b.ev_b[i]);
    }
    b.ev_kind.clear();
    b.ev_a.clear();
    b.ev_b.clear();
    return MITHRA_OK;
}

// sync_stream, then report (and clear) the non-finite flags
static mithra_status sync(Batch &b)
{
    mithra_status st = sync_stream(b);
    if (st) return st;
    std::vector<int> flags(b.nsim, 0);
    HIP_TRY(hipMemcpy(flags.data(), b.ar.flags, sizeof(int) * b.nsim, hipMemcpyDeviceToHost));
    for (int s = 0; s < b.nsim; ++s)
        if (flags[s]) {
            HIP_TRY(hipMemset(b.ar.flags, 0, sizeof(int) * b.nsim));
            return fail(MITHRA_ENUMERIC, "sim %d produced a non-finite momentum or diagnostic", s);
        }
    return MITHRA_OK;
}

// ---------------------------------------------------------------------------
// read-back
// ---------------------------------------------------------------------------

static void *mesh_ptr(Batch &b, int s, int which, bool *ok)
{
    const long long st = b.step;
    *ok = true;
    void *base = nullptr;
    if (which <= MITHRA_PHI) base = b.ar.pot[st % 3][which];
    else if (which <= MITHRA_JZ) base = b.ar.J[which - MITHRA_JX];
    else if (which == MITHRA_RHO) base = b.ar.rho[st & 1];
    else if (which >= MITHRA_AX_PREV && which <= MITHRA_PHI_PREV)
        base = b.ar.pot[(st + 2) % 3][which - MITHRA_AX_PREV];
    else if (which == MITHRA_RHO_PREV) base = b.ar.rho[(st + 1) & 1];
    else {
        *ok = false;
        return nullptr;
    }
    return (char *)base + (size_t)b.sd[s].cell0 * b.rs;
}

static mithra_status get_field(Batch &b, int s, int which, double *host)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    if (!host) return fail(MITHRA_EINVAL, "host is NULL");
    mithra_status st = sync_stream(b);
    if (st) return st;
    const SimDev &S = b.sd[s];
    const long long ncell = (long long)S.n[0] * S.n[1] * S.n[2];
    if (which >= MITHRA_EX && which <= MITHRA_BZ) {
        if (!b.d_eb) {
            size_t maxc = 0;
            for (int i = 0; i < b.nsim; ++i)
                maxc = std::max(maxc, (size_t)b.sd[i].n[0] * b.sd[i].n[1] * b.sd[i].n[2]);
            b.d_eb = (double *)dev_alloc(b, sizeof(double) * 6 * maxc, b.mem_tab);
            if (!b.d_eb) return fail(MITHRA_ENOMEM, "device allocation failed");
        }
        if (b.prec == MITHRA_F64) launch_vertex_fields<double>(b.stream, b.d_sims, s, 0, ncell, b.ar, b.d_eb);
        else launch_vertex_fields<float>(b.stream, b.d_sims, s, 0, ncell, b.ar, b.d_eb);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(host, b.d_eb + (size_t)(which - MITHRA_EX) * ncell,
                               sizeof(double) * ncell, hipMemcpyDeviceToHost, b.stream));
        HIP_TRY(hipStreamSynchronize(b.stream));
        return MITHRA_OK;
    }
    bool ok;
    void *src = mesh_ptr(b, s, which, &ok);
    if (!ok) return fail(MITHRA_EINVAL, "unknown field %d", which);
    if (b.rs == 8) {
        HIP_TRY(hipMemcpy(host, src, sizeof(double) * ncell, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(ncell);
        HIP_TRY(hipMemcpy(tmp.data(), src, sizeof(float) * ncell, hipMemcpyDeviceToHost));
        for (long long i = 0; i < ncell; ++i) host[i] = tmp[i];
    }
    return MITHRA_OK;
}

// get_field without any allocation, host or device: E and B are computed, and
// float fields widened, in the library's static scratch a chunk of whole
// z-planes at a time, each chunk copied to its place in the caller's array
static mithra_status get_field_noalloc(Batch &b, int s, int which, double *host)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    if (!host) return fail(MITHRA_EINVAL, "host is NULL");
    mithra_status st = sync_stream(b);
    if (st) return st;
    const SimDev &S = b.sd[s];
    const long long plane = (long long)S.n[0] * S.n[1];
    const long long ncell = plane * S.n[2];
    if (plane > NOALLOC_CELLS)
        return fail(MITHRA_EINVAL,
                    "a z-plane of %lld points exceeds the %lld points of the allocation-free "
                    "read-back's scratch", plane, NOALLOC_CELLS);
    double *scr = (double *)g_scratch_ptr[b.device];
    if (!scr) return fail(MITHRA_ESTATE, "no read-back scratch on device %d", b.device);
    const bool eb = which >= MITHRA_EX && which <= MITHRA_BZ;
    void *src = nullptr;
    if (!eb) {
        bool ok;
        src = mesh_ptr(b, s, which, &ok);
        if (!ok) return fail(MITHRA_EINVAL, "unknown field %d", which);
        if (b.rs == 8) {
            HIP_TRY(hipMemcpyAsync(host, src, sizeof(double) * ncell, hipMemcpyDeviceToHost,
                                   b.stream));
            HIP_TRY(hipStreamSynchronize(b.stream));
            return MITHRA_OK;
        }
    }
    const long long per = (NOALLOC_CELLS / plane) * plane;
    for (long long g0 = 0; g0 < ncell; g0 += per) {
        const long long count = std::min(per, ncell - g0);
        const double *from = scr;
        if (eb) {
            if (b.prec == MITHRA_F64)
                launch_vertex_fields<double>(b.stream, b.d_sims, s, g0, count, b.ar, scr);
            else
                launch_vertex_fields<float>(b.stream, b.d_sims, s, g0, count, b.ar, scr);
            from = scr + (size_t)(which - MITHRA_EX) * count;
        } else {
            launch_to_double(b.stream, (const float *)src + g0, count, scr);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(host + g0, from, sizeof(double) * count, hipMemcpyDeviceToHost,
                               b.stream));
        HIP_TRY(hipStreamSynchronize(b.stream));
    }
    return MITHRA_OK;
}

static mithra_status set_field(Batch &b, int s, int which, const double *host)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    if (!host) return fail(MITHRA_EINVAL, "host is NULL");
    if (which >= MITHRA_EX && which <= MITHRA_BZ)
        return fail(MITHRA_EINVAL, "E and B are derived from the potentials and cannot be set");
    HIP_TRY(hipStreamSynchronize(b.stream));
    const SimDev &S = b.sd[s];
    const long long ncell = (long long)S.n[0] * S.n[1] * S.n[2];
    bool ok;
    void *dst = mesh_ptr(b, s, which, &ok);
    if (!ok) return fail(MITHRA_EINVAL, "unknown field %d", which);
    for (long long i = 0; i < ncell; ++i)
        if (!std::isfinite(host[i])) return fail(MITHRA_EINVAL, "non-finite value at %lld", i);
    if (b.rs == 8) {
        HIP_TRY(hipMemcpy(dst, host, sizeof(double) * ncell, hipMemcpyHostToDevice));
    } else {
        std::vector<float> tmp(host, host + ncell);
        HIP_TRY(hipMemcpy(dst, tmp.data(), sizeof(float) * ncell, hipMemcpyHostToDevice));
    }
    HIP_TRY(mark_sources_dirty(b));
    HIP_TRY(hipStreamSynchronize(b.stream));
    return MITHRA_OK;
}

template <typename R>
static mithra_status get_particles_impl(Batch &b, int s, double *pos, double *u, uint8_t *alive,
                                        int64_t *np_alive)
{
    const SimDev &S = b.sd[s];
    const long long np = S.np, p0 = S.part0;
    const int par = (int)(b.step & 1);
    std::vector<int> key(np), id(np);
    std::vector<R> f[3], uu[3];
    if (np > 0) {
        HIP_TRY(hipMemcpy(key.data(), b.ar.key[par] + p0, sizeof(int) * np, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(id.data(), b.ar.id[par] + p0, sizeof(int) * np, hipMemcpyDeviceToHost));
        for (int a = 0; a < 3; ++a) {
            f[a].resize(np);
            uu[a].resize(np);
            HIP_TRY(hipMemcpy(f[a].data(), (R *)b.ar.off[par][a] + p0, sizeof(R) * np,
                              hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(uu[a].data(), (R *)b.ar.u[par][a] + p0, sizeof(R) * np,
                              hipMemcpyDeviceToHost));
        }
    }
    long long live = 0;
    for (long long i = 0; i < np; ++i) {
        const int p = id[i];
        if (p < 0 || p >= np) return fail(MITHRA_EDEVICE, "corrupt particle id %d", p);
        const int local = key[i] - (int)S.key0;
        const bool al = local >= 0 && local < S.nkeys;
        int c[3] = {0, 0, 0};
        if (al) {
            const int t = local >> 9, l = local & 511;
            c[0] = (t % S.nt[0]) * TILE + (l & 7);
            c[1] = ((t / S.nt[0]) % S.nt[1]) * TILE + ((l >> 3) & 7);
            c[2] = (t / (S.nt[0] * S.nt[1])) * TILE + (l >> 6);
            ++live;
        }
        for (int a = 0; a < 3; ++a) {
            if (pos)
                pos[3 * p + a] = al ? S.origin[a] + ((double)c[a] + (double)f[a][i]) * S.d[a] : NAN;
            if (u) u[3 * p + a] = (double)uu[a][i];
        }
        if (alive) alive[p] = al ? 1 : 0;
    }
    if (np_alive) *np_alive = live;
    return MITHRA_OK;
}

static mithra_status get_particles(Batch &b, int s, double *pos, double *u, uint8_t *alive,
                                   int64_t *np_alive)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    if (!b.committed) return fail(MITHRA_ESTATE, "particles are not on the device yet (run first)");
    mithra_status st = sync_stream(b);
    if (st) return st;
    return b.prec == MITHRA_F64 ? get_particles_impl<double>(b, s, pos, u, alive, np_alive)
                                : get_particles_impl<float>(b, s, pos, u, alive, np_alive);
}

// the binning of the current particle buffer, as the next step reads it
static mithra_status get_bins(Batch &b, int s, int32_t *keys, int32_t *ids, int32_t *starts,
                              int64_t *nkeys)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    if (!b.committed) return fail(MITHRA_ESTATE, "particles are not on the device yet (run first)");
    mithra_status st = sync_stream(b);
    if (st) return st;
    const SimDev &S = b.sd[s];
    const int par = (int)(b.step & 1);
    if (nkeys) *nkeys = S.nkeys;
    if (S.np > 0 && keys) {
        HIP_TRY(hipMemcpy(keys, b.ar.key[par] + S.part0, sizeof(int) * S.np, hipMemcpyDeviceToHost));
        for (long long i = 0; i < S.np; ++i) keys[i] -= (int32_t)S.key0;
    }
    if (S.np > 0 && ids)
        HIP_TRY(hipMemcpy(ids, b.ar.id[par] + S.part0, sizeof(int) * S.np, hipMemcpyDeviceToHost));
    if (starts) {
        HIP_TRY(hipMemcpy(starts, b.ar.offs[par] + S.key0, sizeof(int) * ((size_t)S.nkeys + 2),
                          hipMemcpyDeviceToHost));
        for (long long g = 0; g < (long long)S.nkeys + 2; ++g) starts[g] -= (int32_t)S.part0;
    }
    return MITHRA_OK;
}

static mithra_status get_diag(Batch &b, int s, mithra_diag_row *rows, int64_t cap, int64_t *nrows)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    if (!nrows || (cap > 0 && !rows)) return fail(MITHRA_EINVAL, "rows/nrows is NULL");
    mithra_status st = sync_stream(b);
    if (st) return st;
    HostSim &h = b.hs[s];
    const SimDev &S = b.sd[s];
    long long first = std::max(h.read_step, b.step - (long long)S.ring_cap);
    long long n = std::min<long long>(b.step - first, cap);
    if (n < 0) n = 0;
    std::vector<double> ring((size_t)S.ring_cap * NDIAG);
    if (n > 0)
        HIP_TRY(hipMemcpy(ring.data(), b.ar.ring + S.ring0 * NDIAG,
                          sizeof(double) * NDIAG * S.ring_cap, hipMemcpyDeviceToHost));
    for (long long r = 0; r < n; ++r) {
        const double *v = &ring[(size_t)((first + r) % S.ring_cap) * NDIAG];
        mithra_diag_row &o = rows[r];
        o.step = (int64_t)v[0];
        o.t = v[1];
        o.total_charge = v[2];
        o.continuity_residual = v[3];
        o.power = v[4];
        o.field_energy = v[5];
        o.kinetic_energy = v[6];
        for (int a = 0; a < 3; ++a) {
            o.probe_E[a] = v[7 + a];
            o.probe_B[a] = v[10 + a];
        }
        o.lost = (int64_t)v[13];
        o.nonfinite = (int32_t)v[14];
        o.has_mesh_terms = (int32_t)v[15];
        for (int h = 0; h < 3; ++h) o.bunching[h] = v[16 + h];
        for (int h = 0; h < 3; ++h) o.power_harmonic[h] = v[20 + h];
        for (int e = 0; e < 3; ++e) o.power_extra[e] = v[24 + e];
        o.power_lab = v[27];
        o.z_undulator = v[28];
    }
    h.read_step = first + n;
    *nrows = n;
    return MITHRA_OK;
}

static mithra_status config_diag(Batch &b, int s, const mithra_diag_cfg *cfg)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    if (!cfg) return fail(MITHRA_EINVAL, "cfg is NULL");
    HostSim &h = b.hs[s];
    for (int a = 0; a < 3; ++a)
        if (cfg->probe[a] < 0 || cfg->probe[a] >= h.mesh.n[a])
            return fail(MITHRA_EINVAL, "probe[%d] = %d outside the mesh", a, cfg->probe[a]);
    if (cfg->power_plane_k < 0 || cfg->power_plane_k >= h.mesh.n[2])
        return fail(MITHRA_EINVAL, "power_plane_k outside the mesh");
    if (cfg->mesh_diag_every < 0) return fail(MITHRA_EINVAL, "mesh_diag_every < 0");
    if (cfg->capacity != h.diag.capacity && b.step > 0)
        return fail(MITHRA_ESTATE, "the ring capacity can only change before the first step");
    if (cfg->capacity < 1 || cfg->capacity > (1 << 24))
        return fail(MITHRA_EINVAL, "capacity must be in [1, 2^24]");
    if (cfg->power_spectrum != 0 && cfg->power_spectrum != 1)
        return fail(MITHRA_EINVAL, "power_spectrum must be 0 or 1");
    if (cfg->power_spectrum != h.diag.power_spectrum && b.step > 0)
        return fail(MITHRA_ESTATE, "the power spectrum can only be switched before the first step");
    for (int e = 0; e < 3; ++e)
        if (cfg->extra_planes[e] < -1 || cfg->extra_planes[e] >= h.mesh.n[2])
            return fail(MITHRA_EINVAL, "extra_planes[%d] = %d: -1 or a z index of the mesh", e,
                        cfg->extra_planes[e]);
    HIP_TRY(hipStreamSynchronize(b.stream));
    if (cfg->capacity != h.diag.capacity) {
        // re-lay the rings (no rows exist before the first step); the new
        // rings are in place before anything else changes
        const int old = h.diag.capacity;
        h.diag.capacity = cfg->capacity;
        mithra_status st = relay_diag_arenas(b, false);
        if (st) {
            h.diag.capacity = old;
            return st;
        }
    }
    h.diag = *cfg;
    SimDev &S = b.sd[s];
    S.probe[0] = cfg->probe[0];
    S.probe[1] = cfg->probe[1];
    S.probe[2] = cfg->probe[2];
    S.kp = cfg->power_plane_k;
    S.zu0 = plate_position(h);  // the plate may have moved
    S.mesh_every = cfg->mesh_diag_every;
    S.ring_cap = cfg->capacity;
    S.spec_on = cfg->power_spectrum;
    S.n_extra = 0;
    for (int e = 0; e < 3; ++e)
        if (cfg->extra_planes[e] >= 0) S.kp_extra[S.n_extra++] = cfg->extra_planes[e];
    return build_tables(b);
}

static mithra_status set_spectrum(Batch &b, int s, const double *nu, int32_t nfreq)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    if (!nu || nfreq < 1 || nfreq > MAXF)
        return fail(MITHRA_EINVAL, "need 1..%d normalized frequencies", MAXF);
    for (int f = 0; f < nfreq; ++f)
        if (!(nu[f] > 0.0) || !std::isfinite(nu[f]))
            return fail(MITHRA_EINVAL, "normalized frequency %d = %g must be positive and finite", f,
                        nu[f]);
    if (b.step > 0)
        return fail(MITHRA_ESTATE, "the spectrum frequencies can only change before the first step");
    HIP_TRY(hipStreamSynchronize(b.stream));
    HostSim &h = b.hs[s];
    const int old_n = h.nfreq;
    double old_f[MAXF];
    std::memcpy(old_f, h.fnu, sizeof old_f);
    h.nfreq = nfreq;
    for (int f = 0; f < MAXF; ++f) h.fnu[f] = f < nfreq ? nu[f] : 0.0;
    mithra_status st = relay_diag_arenas(b, true);
    if (st) {
        h.nfreq = old_n;
        std::memcpy(h.fnu, old_f, sizeof old_f);
        return st;
    }
    for (int i = 0; i < b.nsim; ++i) {
        b.sd[i].nfreq = b.hs[i].nfreq;
        std::memcpy(b.sd[i].fnu, b.hs[i].fnu, sizeof b.sd[i].fnu);
    }
    return build_tables(b);
}

static mithra_status get_spectrum(Batch &b, int s, int64_t first, int64_t count, double *rest,
                                  double *lab)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    if (count < 0 || (count > 0 && (!rest || !lab)))
        return fail(MITHRA_EINVAL, "count < 0 or rest/lab NULL");
    mithra_status st = sync_stream(b);
    if (st) return st;
    const SimDev &S = b.sd[s];
    if (!S.spec_on) return fail(MITHRA_ESTATE, "the power spectrum is off (mithra_diag_cfg.power_spectrum)");
    const long long lo = std::max(0LL, b.step - (long long)S.ring_cap);
    if (first < lo || first + count > b.step)
        return fail(MITHRA_EINVAL, "steps %lld..%lld not in the kept rows %lld..%lld",
                    (long long)first, (long long)(first + count - 1), lo, b.step - 1);
    if (count == 0) return MITHRA_OK;
    const int nf = S.nfreq;
    std::vector<double> ring((size_t)S.ring_cap * 2 * nf);
    HIP_TRY(hipMemcpy(ring.data(), b.ar.srow + S.srow0, sizeof(double) * ring.size(),
                      hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < count; ++r) {
        const double *v = &ring[(size_t)((first + r) % S.ring_cap) * 2 * nf];
        std::memcpy(rest + r * nf, v, sizeof(double) * nf);
        std::memcpy(lab + r * nf, v + nf, sizeof(double) * nf);
    }
    return MITHRA_OK;
}

// checks of a wave's parameters (the seed and the optical undulator)
static mithra_status check_wave(const mithra_seed *w, const char *what)
{
    const double v[] = {w->amplitude, w->polarization[0], w->polarization[1], w->frequency,
                        w->t0, w->tau, w->cep, w->z_ref};
    for (double x : v)
        if (!std::isfinite(x)) return fail(MITHRA_EINVAL, "%s: non-finite value", what);
    if (!(w->tau > 0.0)) return fail(MITHRA_EINVAL, "%s: tau must be > 0", what);
    if (w->frequency < 0.0) return fail(MITHRA_EINVAL, "%s: frequency must be >= 0", what);
    if (w->signal < MITHRA_SIGNAL_NEUMANN || w->signal > MITHRA_SIGNAL_FLAT_TOP)
        return fail(MITHRA_EINVAL, "%s: unknown signal %d", what, w->signal);
    return MITHRA_OK;
}

static mithra_status set_seed(Batch &b, int s, const mithra_seed *seed)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    HostSim &h = b.hs[s];
    mithra_seed z{};
    if (seed && seed->amplitude != 0.0) {
        mithra_status st = check_wave(seed, "seed");
        if (st) return st;
        if (h.mesh.bc[2] == MITHRA_BC_PERIODIC)
            return fail(MITHRA_EINVAL, "seed: the z axis must be absorbing (the wave enters at z_min)");
        z = *seed;
    }
    HIP_TRY(hipStreamSynchronize(b.stream));
    const std::vector<int> before = seed_beam_sims(b);
    h.seed = z;
    fill_seed(h, b.sd[s]);
    if (seed_beam_sims(b) != before) drop_graph(b);
    // the per-simulation block on the device is read at every launch
    HIP_TRY(hipMemcpyAsync(b.d_sims + s, &b.sd[s], sizeof(SimDev), hipMemcpyHostToDevice, b.stream));
    HIP_TRY(hipStreamSynchronize(b.stream));
    return MITHRA_OK;
}

static mithra_status set_optical(Batch &b, int s, const mithra_seed *wave)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    HostSim &h = b.hs[s];
    mithra_seed z{};
    if (wave && wave->amplitude != 0.0) {
        mithra_status st = check_wave(wave, "optical undulator");
        if (st) return st;
        z = *wave;
    }
    HIP_TRY(hipStreamSynchronize(b.stream));
    const int before = any_optical(b);
    h.optical = z;
    fill_optical(h, b.sd[s]);
    // the captured step launches the push variant chosen at capture
    if (any_optical(b) != before) drop_graph(b);
    HIP_TRY(hipMemcpyAsync(b.d_sims + s, &b.sd[s], sizeof(SimDev), hipMemcpyHostToDevice, b.stream));
    HIP_TRY(hipStreamSynchronize(b.stream));
    return MITHRA_OK;
}

static mithra_status check_beam(const mithra_beam *beam, const char *what)
{
    if (!beam) return fail(MITHRA_EINVAL, "%s: beam is NULL", what);
    if (beam->type != MITHRA_BEAM_PLANE && beam->type != MITHRA_BEAM_GAUSSIAN)
        return fail(MITHRA_EINVAL, "%s: unknown beam type %d", what, beam->type);
    if (beam->type == MITHRA_BEAM_GAUSSIAN) {
        for (int a = 0; a < 2; ++a)
            if (!std::isfinite(beam->rayleigh[a]) || !(beam->rayleigh[a] > 0.0))
                return fail(MITHRA_EINVAL, "%s: Rayleigh lengths must be finite and > 0", what);
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(beam->focus[a]))
                return fail(MITHRA_EINVAL, "%s: the focus must be finite", what);
    }
    return MITHRA_OK;
}

static mithra_status set_optical_beam(Batch &b, int s, const mithra_beam *beam)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    mithra_status st = check_beam(beam, "optical beam");
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(b.stream));
    HostSim &h = b.hs[s];
    h.beam = *beam;
    fill_optical(h, b.sd[s]);
    HIP_TRY(hipMemcpyAsync(b.d_sims + s, &b.sd[s], sizeof(SimDev), hipMemcpyHostToDevice, b.stream));
    HIP_TRY(hipStreamSynchronize(b.stream));
    return MITHRA_OK;
}

static mithra_status set_seed_beam(Batch &b, int s, const mithra_beam *beam)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    mithra_status st = check_beam(beam, "seed beam");
    if (st) return st;
    HostSim &h = b.hs[s];
    HIP_TRY(hipStreamSynchronize(b.stream));
    if (beam->type == MITHRA_BEAM_GAUSSIAN && !h.seed_corr) {
        // corrections of A_x and A_y on planes 2 and 3, every column
        h.seed_corr = (double *)dev_alloc(b, sizeof(double) * 4 * (size_t)h.mesh.n[0] * h.mesh.n[1],
                                          b.mem_fixed);
        if (!h.seed_corr) return fail(MITHRA_ENOMEM, "device allocation of the seed corrections failed");
    }
    const std::vector<int> before = seed_beam_sims(b);
    h.seed_beam = *beam;
    fill_seed(h, b.sd[s]);
    if (seed_beam_sims(b) != before) drop_graph(b);
    HIP_TRY(hipMemcpyAsync(b.d_sims + s, &b.sd[s], sizeof(SimDev), hipMemcpyHostToDevice, b.stream));
    HIP_TRY(hipStreamSynchronize(b.stream));
    return MITHRA_OK;
}

template <typename R>
static mithra_status upload_background(Batch &b, HostSim &h, const double *rho)
{
    const size_t ncell = (size_t)h.mesh.n[0] * h.mesh.n[1] * h.mesh.n[2];
    std::vector<R> v(ncell);
    for (size_t c = 0; c < ncell; ++c) v[c] = (R)rho[c];
    HIP_TRY(hipMemcpy(h.bg, v.data(), sizeof(R) * ncell, hipMemcpyHostToDevice));
    return MITHRA_OK;
}

static mithra_status set_background(Batch &b, int s, const double *rho)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    HostSim &h = b.hs[s];
    const size_t ncell = (size_t)h.mesh.n[0] * h.mesh.n[1] * h.mesh.n[2];
    if (rho)
        for (size_t c = 0; c < ncell; ++c)
            if (!std::isfinite(rho[c]))
                return fail(MITHRA_EINVAL, "background: value %zu is not finite", c);
    HIP_TRY(hipStreamSynchronize(b.stream));
    if (rho && !h.bg) {
        h.bg = dev_alloc(b, b.rs * ncell, b.mem_fixed);
        h.rho_bg = h.bg ? dev_alloc(b, b.rs * ncell, b.mem_fixed) : nullptr;
        if (!h.bg || !h.rho_bg) {
            h.bg = h.rho_bg = nullptr;  // released with the batch
            return fail(MITHRA_ENOMEM, "device allocation of the background failed");
        }
    }
    if (rho) {
        mithra_status st = b.prec == MITHRA_F64 ? upload_background<double>(b, h, rho)
                                                : upload_background<float>(b, h, rho);
        if (st) return st;
    }
    const std::vector<int> before = background_sims(b);
    h.has_bg = rho != nullptr;
    SimDev &S = b.sd[s];
    S.bg = h.has_bg ? h.bg : nullptr;
    S.rho_bg = h.has_bg ? h.rho_bg : nullptr;
    if (background_sims(b) != before) drop_graph(b);
    HIP_TRY(hipMemcpyAsync(b.d_sims + s, &S, sizeof(SimDev), hipMemcpyHostToDevice, b.stream));
    HIP_TRY(hipStreamSynchronize(b.stream));
    return MITHRA_OK;
}

static mithra_status get_info(Batch &b, int s, mithra_info *info)
{
    if (s < 0 || s >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", s);
    if (!info) return fail(MITHRA_EINVAL, "info is NULL");
    const HostSim &h = b.hs[s];
    info->dt = h.dt;
    info->dtb = h.dtb;
    info->nsfd_A = h.A;
    info->gamma0 = h.gamma0;
    info->beta0 = h.beta0;
    info->B0 = h.B0;
    info->ku = h.ku;
    info->step = b.step;
    info->np = (int64_t)h.alive.size();
    info->device_bytes = (int64_t)b.bytes;
    info->stencil_tile[0] = b.tile_x;
    info->stencil_tile[1] = b.tile_y;
    info->stencil_tile[2] = b.kz;
    info->precision = b.prec;
    for (int a = 0; a < 3; ++a) info->particle_brick[a] = b.brick[a];
    info->pad = 0;
    return MITHRA_OK;
}

// ---------------------------------------------------------------------------
// autotuner: the stencil rewrites level s+1 from levels s and s-1, so timing
// it repeatedly leaves the state unchanged.
// ---------------------------------------------------------------------------

// The brick shape of the push and the deposit: each candidate times trials
// launches of the push followed by the deposit on the simulation's current
// particles.  Those kernels change the particle buffer in place and write J,
// rho, the bin counts, the error flags and the per-tile flags (occupancy,
// active, dirty), so these are copied aside first and put back after every
// trial: each trial does a step's work (with the occupancy flags left as the
// first trial leaves them, the later pushes would find every tile empty).
// During the trials the dirty flags are cleared, as in a running simulation
// where the tiles away from the bunch hold zero sources and are skipped; the
// copies put back at the end restore them.  The results of a step never
// depend on the brick shape.
template <typename R>
static mithra_status tune_bricks(Batch &b, int trials)
{
    static const int shapes[][3] = {{2, 2, 2}, {4, 4, 2}, {4, 4, 4}, {8, 8, 2}, {8, 4, 4},
                                    {4, 4, 8}, {8, 8, 4}, {2, 2, 16}, {16, 16, 2}, {32, 32, 2}};
    HIP_TRY(hipStreamSynchronize(b.stream));
    const long long N = b.total_particles, M = b.total_cells;
    const int par = (int)(b.step & 1), dst = par ^ 1;
    struct Span {
        void *p;
        size_t bytes;
    };
    std::vector<Span> keep = {{b.ar.key[par], sizeof(int) * N}, {b.ar.rho[dst], sizeof(R) * M},
                              {b.ar.flags, sizeof(int) * b.nsim}};
    for (int a = 0; a < 3; ++a) {
        keep.push_back({b.ar.off[par][a], sizeof(R) * N});
        keep.push_back({b.ar.u[par][a], sizeof(R) * N});
        keep.push_back({b.ar.J[a], sizeof(R) * M});
    }
    const size_t tb = sizeof(int) * std::max(b.n_tiles, 1);
    for (int *f : {b.ar.pocc[0], b.ar.pocc[1], b.ar.tact, b.ar.jdirty, b.ar.rdirty[0],
                   b.ar.rdirty[1]})
        keep.push_back({f, tb});
    std::vector<Batch::Block> scratch;
    std::vector<void *> copy;
    for (const Span &k : keep) {
        void *c = dev_alloc(b, std::max<size_t>(k.bytes, 1), scratch);
        if (!c) {
            dev_free_all(b, scratch);
            return MITHRA_OK;  // no room to tune: keep the current shape
        }
        copy.push_back(c);
        HIP_TRY(hipMemcpyAsync(c, k.p, k.bytes, hipMemcpyDeviceToDevice, b.stream));
    }
    auto restore = [&](bool trial) -> hipError_t {
        hipError_t e = hipSuccess;
        for (size_t i = 0; i < keep.size() && e == hipSuccess; ++i)
            e = hipMemcpyAsync(keep[i].p, copy[i], keep[i].bytes, hipMemcpyDeviceToDevice, b.stream);
        if (e == hipSuccess) e = hipMemsetAsync(b.ar.counts, 0, sizeof(int) * b.total_keys, b.stream);
        for (int *f : {b.ar.jdirty, b.ar.rdirty[0], b.ar.rdirty[1]})
            if (trial && e == hipSuccess) e = hipMemsetAsync(f, 0, tb, b.stream);
        return e;
    };
    int maxt[3] = {1, 1, 1};
    for (int s = 0; s < b.nsim; ++s)
        for (int a = 0; a < 3; ++a) maxt[a] = std::max(maxt[a], b.sd[s].nt[a]);
    hipEvent_t e0 = new_event(), e1 = new_event();
    struct Cand {
        int c[3];
        Brick *d;
        int n;
        float ms;
    };
    std::vector<Cand> cands;
    std::vector<Brick> table;
    // the fixed shapes that fit in some grid, then whole tile layers of the
    // largest grid, one, two and four deep
    std::vector<std::array<int, 3>> cand_shapes;
    for (const auto &sh : shapes)
        if (sh[0] <= maxt[0] && sh[1] <= maxt[1] && sh[2] <= maxt[2])
            cand_shapes.push_back({sh[0], sh[1], sh[2]});
    for (int d : {1, 2, 4}) {
        const std::array<int, 3> w = {maxt[0], maxt[1], std::min(d, maxt[2])};
        if (std::find(cand_shapes.begin(), cand_shapes.end(), w) == cand_shapes.end())
            cand_shapes.push_back(w);
    }
    for (const auto &sh : cand_shapes) {
        Cand k;
        for (int a = 0; a < 3; ++a) k.c[a] = sh[a];
        brick_table(b, k.c, table);
        k.d = (Brick *)dev_alloc(b, table.size() * sizeof(Brick), scratch);
        if (!k.d) continue;
        HIP_TRY(hipMemcpyAsync(k.d, table.data(), table.size() * sizeof(Brick),
                               hipMemcpyHostToDevice, b.stream));
        HIP_TRY(hipStreamSynchronize(b.stream));  // the host table is refilled next
        k.n = (int)table.size();
        k.ms = 1e30f;
        cands.push_back(k);
    }
    // two passes, the second in reverse order, each candidate keeping its
    // best trial, so that a slow spell of the device does not decide
    for (int pass = 0; pass < 2; ++pass) {
        for (size_t q = 0; q < cands.size(); ++q) {
            Cand &k = cands[pass ? cands.size() - 1 - q : q];
            for (int t = 0; t < trials + 1; ++t) {  // the first is a warm-up
                HIP_TRY(restore(true));
                HIP_TRY(hipEventRecord(e0, b.stream));
                launch_push<R>(b.stream, b.d_sims, k.d, k.n, brick_shape(k.c), b.ar,
                               any_optical(b));
                launch_deposit<R>(b.stream, b.d_sims, k.d, k.n, brick_shape(k.c), b.ar, 0);
                HIP_TRY(hipEventRecord(e1, b.stream));
                HIP_TRY(hipEventSynchronize(e1));
                HIP_TRY(hipGetLastError());
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (t > 0) k.ms = std::min(k.ms, ms);
            }
        }
    }
    float best = 1e30f;
    int pick[3] = {b.brick[0], b.brick[1], b.brick[2]};
    for (const Cand &k : cands)
        if (k.ms < best) {
            best = k.ms;
            for (int a = 0; a < 3; ++a) pick[a] = k.c[a];
        }
    HIP_TRY(restore(false));
    HIP_TRY(hipStreamSynchronize(b.stream));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dev_free_all(b, scratch);
    for (int a = 0; a < 3; ++a) b.brick[a] = pick[a];
    return MITHRA_OK;
}

template <typename R>
static mithra_status tune_impl(Batch &b, int trials)
{
    static const int shapes[][2] = {{64, 4}, {32, 8}, {128, 2}, {64, 2}, {32, 4}, {16, 16},
                                    {256, 1}, {128, 1}, {128, 4}, {256, 2}, {64, 8}};
    static const int kzs[] = {16, 32, 64, 128, 256};
    int maxn[3] = {0, 0, 0};
    for (int s = 0; s < b.nsim; ++s)
        for (int a = 0; a < 3; ++a) maxn[a] = std::max(maxn[a], b.sd[s].n[a]);
    hipEvent_t e0 = new_event(), e1 = new_event();
    int bx = b.tile_x, by = b.tile_y, bk = b.kz;
    struct Cand {
        int tx, ty, kz, fx, n;
        int4 *items;
        float ms;
    };
    std::vector<Cand> cands;
    std::vector<int4> items;
    std::vector<Batch::Block> scratch;
    for (auto &sh : shapes) {
        if (sh[0] > 2 * maxn[0] && sh[0] > 16) continue;
        for (int kz : kzs) {
            if (kz > 2 * maxn[2]) continue;
            stencil_items(b, sh[0], sh[1], kz, items);
            int4 *d = (int4 *)dev_alloc(b, items.size() * sizeof(int4), scratch);
            if (!d) continue;
            HIP_TRY(hipMemcpyAsync(d, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice,
                                   b.stream));
            cands.push_back({sh[0], sh[1], kz, x_faces_fusable(b, sh[0]) ? 1 : 0,
                             (int)items.size(), d, 1e30f});
        }
    }
    // two passes, the second in reverse order; each candidate keeps its best
    for (int pass = 0; pass < 2; ++pass) {
        for (size_t q = 0; q < cands.size(); ++q) {
            Cand &c = cands[pass ? cands.size() - 1 - q : q];
            launch_stencil<R>(b.stream, b.d_sims, c.items, c.n, b.ar, c.tx, c.ty, c.kz, c.fx);
            HIP_TRY(hipEventRecord(e0, b.stream));
            for (int t = 0; t < trials; ++t)
                launch_stencil<R>(b.stream, b.d_sims, c.items, c.n, b.ar, c.tx, c.ty, c.kz, c.fx);
            HIP_TRY(hipEventRecord(e1, b.stream));
            HIP_TRY(hipEventSynchronize(e1));
            HIP_TRY(hipGetLastError());
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            c.ms = std::min(c.ms, ms);
        }
    }
    float best = 1e30f;
    for (const Cand &c : cands)
        if (c.ms < best) {
            best = c.ms;
            bx = c.tx;
            by = c.ty;
            bk = c.kz;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_TRY(hipStreamSynchronize(b.stream));
    dev_free_all(b, scratch);
    b.tile_x = bx;
    b.tile_y = by;
    b.kz = bk;
    if (b.total_particles > 0) {
        mithra_status st = tune_bricks<R>(b, trials);
        if (st) return st;
    }
    return build_tables(b);
}

static mithra_status tune(Batch &b, int trials)
{
    if (trials < 1) return fail(MITHRA_EINVAL, "trial_steps must be >= 1");
    HIP_TRY(hipSetDevice(b.device));
    if (!b.committed) {
        mithra_status st = commit(b);
        if (st) return st;
    }
    return b.prec == MITHRA_F64 ? tune_impl<double>(b, trials) : tune_impl<float>(b, trials);
}

// the tuner's choice set directly (nothing is timed)
static mithra_status set_shapes(Batch &b, const int32_t *tile, const int32_t *brick)
{
    if (!tile || !brick) return fail(MITHRA_EINVAL, "stencil_tile and particle_brick must not be NULL");
    if (!stencil_shape_supported(tile[0], tile[1]))
        return fail(MITHRA_EINVAL, "stencil tile %dx%d is not one of the built shapes", tile[0], tile[1]);
    if (tile[2] < 1) return fail(MITHRA_EINVAL, "z planes per stencil block must be >= 1");
    if (brick[0] < 1 || brick[1] < 1 || brick[2] < 1)
        return fail(MITHRA_EINVAL, "brick sides must be >= 1");
    HIP_TRY(hipSetDevice(b.device));
    b.tile_x = tile[0];
    b.tile_y = tile[1];
    b.kz = tile[2];
    for (int a = 0; a < 3; ++a) b.brick[a] = brick[a];
    return b.committed ? build_tables(b) : MITHRA_OK;  // else the commit builds them
}

// ---------------------------------------------------------------------------
// checkpoint
// ---------------------------------------------------------------------------

struct SpecTrailer {
    int64_t step0;
    int32_t nfreq, pad;
    double fnu[MAXF];
};

struct StateHeader {
    char magic[8];
    int32_t version, prec, n[3], pad;
    int64_t step, np, ncell;
};

template <typename R>
static mithra_status get_state_impl(Batch &b, void *blob, size_t *bytes)
{
    const SimDev &S = b.sd[0];
    const long long ncell = (long long)S.n[0] * S.n[1] * S.n[2];
    const long long np = S.np;
    const size_t mesh_bytes = (size_t)ncell * sizeof(R);
    // potentials at levels s-1 and s, J (3), rho (2), particles in id order:
    // alive (1 byte), cell (3 int), offset (3 R), u (3 R); then (version 3)
    // the spectrum's start step, frequency count and normalized frequencies
    // and its running DFT, 8 doubles per plane point and frequency
    const HostSim &h = b.hs[0];
    const size_t spec_bytes = sizeof(double) * (size_t)S.n[0] * S.n[1] * SPEC_PER_FREQ * h.nfreq;
    const size_t part_bytes = (size_t)np * (1 + 3 * sizeof(int) + 6 * sizeof(R));
    const size_t trail_bytes = sizeof(SpecTrailer);
    const size_t need = sizeof(StateHeader) + mesh_bytes * (8 + 3 + 2) + part_bytes + trail_bytes +
                        spec_bytes;
    if (!blob) {
        *bytes = need;
        return MITHRA_OK;
    }
    if (*bytes < need) return fail(MITHRA_EINVAL, "blob too small: need %zu bytes", need);
    mithra_status st = sync_stream(b);
    if (st) return st;
    char *w = (char *)blob;
    StateHeader hd;
    std::memset(&hd, 0, sizeof hd);
    std::memcpy(hd.magic, "MITHRA1", 8);
    hd.version = 3;
    hd.prec = b.prec;
    for (int a = 0; a < 3; ++a) hd.n[a] = S.n[a];
    hd.step = b.step;
    hd.np = np;
    hd.ncell = ncell;
    std::memcpy(w, &hd, sizeof hd);
    w += sizeof hd;
    const long long s = b.step;
    const size_t off = (size_t)S.cell0 * sizeof(R);
    for (int c = 0; c < 4; ++c) {
        HIP_TRY(hipMemcpy(w, (char *)b.ar.pot[(s + 2) % 3][c] + off, mesh_bytes, hipMemcpyDeviceToHost));
        w += mesh_bytes;
        HIP_TRY(hipMemcpy(w, (char *)b.ar.pot[s % 3][c] + off, mesh_bytes, hipMemcpyDeviceToHost));
        w += mesh_bytes;
    }
    for (int c = 0; c < 3; ++c) {
        HIP_TRY(hipMemcpy(w, (char *)b.ar.J[c] + off, mesh_bytes, hipMemcpyDeviceToHost));
        w += mesh_bytes;
    }
    HIP_TRY(hipMemcpy(w, (char *)b.ar.rho[s & 1] + off, mesh_bytes, hipMemcpyDeviceToHost));
    w += mesh_bytes;
    HIP_TRY(hipMemcpy(w, (char *)b.ar.rho[(s + 1) & 1] + off, mesh_bytes, hipMemcpyDeviceToHost));
    w += mesh_bytes;
    // particles
    const int par = (int)(s & 1);
    std::vector<int> key(np), id(np);
    std::vector<R> f[3], uu[3];
    if (np > 0) {
        HIP_TRY(hipMemcpy(key.data(), b.ar.key[par] + S.part0, sizeof(int) * np, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(id.data(), b.ar.id[par] + S.part0, sizeof(int) * np, hipMemcpyDeviceToHost));
        for (int a = 0; a < 3; ++a) {
            f[a].resize(np);
            uu[a].resize(np);
            HIP_TRY(hipMemcpy(f[a].data(), (R *)b.ar.off[par][a] + S.part0, sizeof(R) * np,
                              hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(uu[a].data(), (R *)b.ar.u[par][a] + S.part0, sizeof(R) * np,
                              hipMemcpyDeviceToHost));
        }
    }
    unsigned char *al = (unsigned char *)w;
    int *cell = (int *)(w + np);
    R *fr = (R *)(w + np + 3 * sizeof(int) * np);
    R *mo = fr + 3 * np;
    for (long long i = 0; i < np; ++i) {
        const int p = id[i];
        const int local = key[i] - (int)S.key0;
        const bool a_ = local >= 0 && local < S.nkeys;
        al[p] = a_ ? 1 : 0;
        int c[3] = {0, 0, 0};
        if (a_) {
            const int t = local >> 9, l = local & 511;
            c[0] = (t % S.nt[0]) * TILE + (l & 7);
            c[1] = ((t / S.nt[0]) % S.nt[1]) * TILE + ((l >> 3) & 7);
            c[2] = (t / (S.nt[0] * S.nt[1])) * TILE + (l >> 6);
        }
        for (int a = 0; a < 3; ++a) {
            cell[3 * p + a] = c[a];
            fr[3 * p + a] = f[a][i];
            mo[3 * p + a] = uu[a][i];
        }
    }
    SpecTrailer tr;
    std::memset(&tr, 0, sizeof tr);
    tr.step0 = h.step0;
    tr.nfreq = h.nfreq;
    std::memcpy(tr.fnu, h.fnu, sizeof tr.fnu);
    std::memcpy(w + part_bytes, &tr, sizeof tr);
    HIP_TRY(hipMemcpy(w + part_bytes + trail_bytes, b.ar.spec + S.spec0, spec_bytes,
                      hipMemcpyDeviceToHost));
    *bytes = need;
    return MITHRA_OK;
}

template <typename R>
static mithra_status set_state_impl(Batch &b, const void *blob, size_t bytes)
{
    SimDev &S0 = b.sd[0];
    const long long ncell = (long long)S0.n[0] * S0.n[1] * S0.n[2];
    if (bytes < sizeof(StateHeader)) return fail(MITHRA_EINVAL, "blob too small");
    StateHeader hd;
    std::memcpy(&hd, blob, sizeof hd);
    if (std::memcmp(hd.magic, "MITHRA1", 8) != 0 || hd.version < 1 || hd.version > 3)
        return fail(MITHRA_EINVAL, "not a state blob of this library");
    if (hd.prec != b.prec || hd.n[0] != S0.n[0] || hd.n[1] != S0.n[1] || hd.n[2] != S0.n[2])
        return fail(MITHRA_EINVAL, "state belongs to another mesh or precision");
    if (!b.hs[0].loaded)
        return fail(MITHRA_ESTATE, "load particles once (any) before restoring a state: q and m come from that call");
    const long long np = hd.np;
    if (hd.step < 0 || np < 0 || np > MAX_PARTICLES)
        return fail(MITHRA_EINVAL, "corrupt state blob (step %lld, %lld particles)",
                    (long long)hd.step, np);
    const size_t mesh_bytes = (size_t)ncell * sizeof(R);
    const size_t npl = (size_t)S0.n[0] * S0.n[1];
    const size_t part_bytes = (size_t)np * (1 + 3 * sizeof(int) + 6 * sizeof(R));
    // the plane spectrum: version 3 carries its start step and frequencies,
    // which must be the simulation's; version 2 carries the harmonics 1, 2, 3
    // from step 0, kept when the simulation samples exactly those; version 1
    // has none.  Without one, the spectrum restarts at the restored step.
    HostSim &h = b.hs[0];
    const bool harmonics = h.nfreq == 3 && h.fnu[0] == 1.0 && h.fnu[1] == 2.0 && h.fnu[2] == 3.0;
    size_t trail_bytes = 0, spec_bytes = 0, spec_keep = 0;
    SpecTrailer tr;
    std::memset(&tr, 0, sizeof tr);
    if (hd.version == 3) {
        trail_bytes = sizeof tr;
        if (bytes < sizeof(StateHeader) + mesh_bytes * 13 + part_bytes + trail_bytes)
            return fail(MITHRA_EINVAL, "blob truncated");
        std::memcpy(&tr, (const char *)blob + sizeof hd + mesh_bytes * 13 + part_bytes, sizeof tr);
        if (tr.nfreq != h.nfreq || std::memcmp(tr.fnu, h.fnu, sizeof tr.fnu) != 0)
            return fail(MITHRA_EINVAL, "state blob: its spectrum frequencies differ from the "
                                       "simulation's (set them with mithra_set_spectrum first)");
        if (tr.step0 < 0 || tr.step0 > hd.step)
            return fail(MITHRA_EINVAL, "corrupt state blob (spectrum start %lld)", (long long)tr.step0);
        spec_bytes = spec_keep = sizeof(double) * npl * SPEC_PER_FREQ * h.nfreq;
    } else if (hd.version == 2) {
        spec_bytes = sizeof(double) * npl * 24;
        spec_keep = harmonics ? spec_bytes : 0;
    }
    const size_t need = sizeof(StateHeader) + mesh_bytes * 13 + part_bytes + trail_bytes + spec_bytes;
    if (bytes < need) return fail(MITHRA_EINVAL, "blob truncated");
    const char *r = (const char *)blob + sizeof hd + mesh_bytes * 13;
    const unsigned char *al = (const unsigned char *)r;
    const int *cell = (const int *)(r + np);
    const R *fr = (const R *)(r + np + 3 * sizeof(int) * np);
    const R *mo = fr + 3 * np;
    // a live particle's cell indexes the bins and the mesh: check every one
    // before anything changes
    for (long long i = 0; i < np; ++i) {
        if (al[i] > 1) return fail(MITHRA_EINVAL, "corrupt state blob (particle %lld)", i);
        if (!al[i]) continue;
        for (int a = 0; a < 3; ++a) {
            const double f = (double)fr[3 * i + a], m = (double)mo[3 * i + a];
            if (cell[3 * i + a] < 2 || cell[3 * i + a] > S0.n[a] - 3 || !(f >= 0.0 && f <= 1.0) ||
                !std::isfinite(m))
                return fail(MITHRA_EINVAL, "corrupt state blob (particle %lld)", i);
        }
    }
    HIP_TRY(hipStreamSynchronize(b.stream));
    // particles first (commit re-lays the arenas at the restored step)
    h.alive.assign(al, al + np);
    h.cell.assign(cell, cell + 3 * np);
    h.frac.resize(3 * np);
    h.mom.resize(3 * np);
    for (long long i = 0; i < 3 * np; ++i) {
        h.frac[i] = (double)fr[i];
        h.mom[i] = (double)mo[i];
    }
    b.step = hd.step;
    mithra_status st = commit_impl<R>(b);
    if (st) return st;
    // fields (overwrite the rho^{s+1/2} and J^s = 0 written by the commit)
    const char *w = (const char *)blob + sizeof hd;
    const long long s = b.step;
    const size_t off = (size_t)S0.cell0 * sizeof(R);
    for (int c = 0; c < 4; ++c) {
        HIP_TRY(hipMemcpy((char *)b.ar.pot[(s + 2) % 3][c] + off, w, mesh_bytes, hipMemcpyHostToDevice));
        w += mesh_bytes;
        HIP_TRY(hipMemcpy((char *)b.ar.pot[s % 3][c] + off, w, mesh_bytes, hipMemcpyHostToDevice));
        w += mesh_bytes;
    }
    for (int c = 0; c < 3; ++c) {
        HIP_TRY(hipMemcpy((char *)b.ar.J[c] + off, w, mesh_bytes, hipMemcpyHostToDevice));
        w += mesh_bytes;
    }
    HIP_TRY(hipMemcpy((char *)b.ar.rho[s & 1] + off, w, mesh_bytes, hipMemcpyHostToDevice));
    w += mesh_bytes;
    HIP_TRY(hipMemcpy((char *)b.ar.rho[(s + 1) & 1] + off, w, mesh_bytes, hipMemcpyHostToDevice));
    if (spec_keep) {
        HIP_TRY(hipMemcpy(b.ar.spec + S0.spec0,
                          (const char *)blob + sizeof hd + mesh_bytes * 13 + part_bytes + trail_bytes,
                          spec_keep, hipMemcpyHostToDevice));
        h.step0 = hd.version == 3 ? tr.step0 : 0;
        S0.step0 = h.step0;
        HIP_TRY(hipMemcpyAsync(b.d_sims, &S0, sizeof(SimDev), hipMemcpyHostToDevice, b.stream));
    }
    HIP_TRY(mark_sources_dirty(b));
    HIP_TRY(hipStreamSynchronize(b.stream));
    h.read_step = s;
    return MITHRA_OK;
}

}  // namespace mithra

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

using namespace mithra;

struct mithra_sim {
    Batch *b;
};
struct mithra_batch {
    Batch *b;
};

extern "C" {

const char *mithra_last_error(void) { return g_err.c_str(); }

mithra_status mithra_set_allocator(void *(*alloc)(size_t, void *), void (*release)(void *, void *),
                                   void *ctx)
{
    if ((alloc == nullptr) != (release == nullptr))
        return fail(MITHRA_EINVAL, "alloc and release must both be set or both be NULL");
    g_alloc = alloc;
    g_free = release;
    g_alloc_ctx = ctx;
    return MITHRA_OK;
}

mithra_status mithra_create(const mithra_mesh *mesh, const mithra_undulator *und,
                            mithra_precision prec, void *stream, mithra_sim **out)
{
    if (!out) return fail(MITHRA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mesh || !und) return fail(MITHRA_EINVAL, "mesh and undulator must not be NULL");
    Batch *b = nullptr;
    mithra_status st = create_batch(1, mesh, und, prec, stream, &b);
    if (st) return st;
    *out = new mithra_sim{b};
    return MITHRA_OK;
}

mithra_status mithra_set_particles(mithra_sim *sim, int64_t np, const double *pos, const double *u,
                                   double q_macro, double m_macro)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    Batch &b = *sim->b;
    HIP_TRY(hipSetDevice(b.device));
    mithra_status st = stage_particles(b.hs[0], 0, np, pos, u, q_macro, m_macro);
    if (st) return st;
    return commit(b);
}

mithra_status mithra_config_diag(mithra_sim *sim, const mithra_diag_cfg *cfg)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return config_diag(*sim->b, 0, cfg);
}

mithra_status mithra_set_spectrum(mithra_sim *sim, const double *nu, int32_t nfreq)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return set_spectrum(*sim->b, 0, nu, nfreq);
}

mithra_status mithra_get_spectrum(mithra_sim *sim, int64_t first_step, int64_t count, double *rest,
                                  double *lab)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return get_spectrum(*sim->b, 0, first_step, count, rest, lab);
}

mithra_status mithra_set_seed(mithra_sim *sim, const mithra_seed *seed)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return set_seed(*sim->b, 0, seed);
}

mithra_status mithra_set_optical_undulator(mithra_sim *sim, const mithra_seed *wave)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return set_optical(*sim->b, 0, wave);
}

mithra_status mithra_set_optical_beam(mithra_sim *sim, const mithra_beam *beam)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return set_optical_beam(*sim->b, 0, beam);
}

mithra_status mithra_set_background(mithra_sim *sim, const double *rho)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return set_background(*sim->b, 0, rho);
}

mithra_status mithra_set_seed_beam(mithra_sim *sim, const mithra_beam *beam)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return set_seed_beam(*sim->b, 0, beam);
}

mithra_status mithra_run(mithra_sim *sim, int64_t nsteps)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    if (!sim->b->hs[0].loaded) return fail(MITHRA_ESTATE, "load particles before running");
    return run(*sim->b, nsteps);
}

mithra_status mithra_sync(mithra_sim *sim)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return sync(*sim->b);
}

mithra_status mithra_get_field(mithra_sim *sim, mithra_field which, double *host)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return get_field(*sim->b, 0, which, host);
}

mithra_status mithra_get_field_noalloc(mithra_sim *sim, mithra_field which, double *host)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return get_field_noalloc(*sim->b, 0, which, host);
}

mithra_status mithra_set_field(mithra_sim *sim, mithra_field which, const double *host)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return set_field(*sim->b, 0, which, host);
}

mithra_status mithra_get_particles(mithra_sim *sim, double *pos, double *u, uint8_t *alive,
                                   int64_t *np_alive)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return get_particles(*sim->b, 0, pos, u, alive, np_alive);
}

mithra_status mithra_get_bins(mithra_sim *sim, int32_t *keys, int32_t *ids, int32_t *starts,
                              int64_t *nkeys)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return get_bins(*sim->b, 0, keys, ids, starts, nkeys);
}

mithra_status mithra_get_diag(mithra_sim *sim, mithra_diag_row *rows, int64_t cap, int64_t *nrows)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return get_diag(*sim->b, 0, rows, cap, nrows);
}

mithra_status mithra_get_info(mithra_sim *sim, mithra_info *info)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return get_info(*sim->b, 0, info);
}

mithra_status mithra_get_state(mithra_sim *sim, void *blob, size_t *bytes)
{
    if (!sim || !bytes) return fail(MITHRA_EINVAL, "sim or bytes is NULL");
    Batch &b = *sim->b;
    if (!b.committed) return fail(MITHRA_ESTATE, "load particles before taking a checkpoint");
    return b.prec == MITHRA_F64 ? get_state_impl<double>(b, blob, bytes)
                                : get_state_impl<float>(b, blob, bytes);
}

mithra_status mithra_set_state(mithra_sim *sim, const void *blob, size_t bytes)
{
    if (!sim || !blob) return fail(MITHRA_EINVAL, "sim or blob is NULL");
    Batch &b = *sim->b;
    HIP_TRY(hipSetDevice(b.device));
    return b.prec == MITHRA_F64 ? set_state_impl<double>(b, blob, bytes)
                                : set_state_impl<float>(b, blob, bytes);
}

mithra_status mithra_set_timing(mithra_sim *sim, int32_t on)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    sim->b->timing = on != 0;
    return MITHRA_OK;
}

mithra_status mithra_get_timing(mithra_sim *sim, double *ms, int64_t *calls, int32_t nkinds,
                                int32_t reset)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    Batch &b = *sim->b;
    mithra_status st = sync_stream(b);
    if (st) return st;
    for (int k = 0; k < std::min<int>(nkinds, NKINDS); ++k) {
        if (ms) ms[k] = b.ms[k];
        if (calls) calls[k] = b.calls[k];
    }
    if (reset)
        for (int k = 0; k < NKINDS; ++k) {
            b.ms[k] = 0.0;
            b.calls[k] = 0;
        }
    return MITHRA_OK;
}

mithra_status mithra_tune(mithra_sim *sim, int32_t trial_steps)
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return tune(*sim->b, trial_steps);
}

mithra_status mithra_set_shapes(mithra_sim *sim, const int32_t stencil_tile[3],
                                const int32_t particle_brick[3])
{
    if (!sim) return fail(MITHRA_EINVAL, "sim is NULL");
    return set_shapes(*sim->b, stencil_tile, particle_brick);
}

void mithra_destroy(mithra_sim *sim)
{
    if (!sim) return;
    destroy_batch(sim->b);
    delete sim;
}

// ---- batch ------------------------------------------------------------------

mithra_status mithra_batch_create(int32_t nsim, const mithra_mesh *meshes,
                                  const mithra_undulator *unds, mithra_precision prec, void *stream,
                                  mithra_batch **out)
{
    if (!out) return fail(MITHRA_EINVAL, "out is NULL");
    *out = nullptr;
    Batch *b = nullptr;
    mithra_status st = create_batch(nsim, meshes, unds, prec, stream, &b);
    if (st) return st;
    *out = new mithra_batch{b};
    return MITHRA_OK;
}

mithra_status mithra_batch_set_particles(mithra_batch *bb, int32_t sim, int64_t np, const double *pos,
                                         const double *u, double q_macro, double m_macro)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    Batch &b = *bb->b;
    if (sim < 0 || sim >= b.nsim) return fail(MITHRA_EINVAL, "sim index %d out of range", sim);
    if (b.step > 0)
        return fail(MITHRA_ESTATE, "batch particles can only be loaded before the first step");
    long long others = 0;
    for (int s = 0; s < b.nsim; ++s)
        if (s != sim) others += (long long)b.hs[s].alive.size();
    if (np > 0 && others + np > MAX_PARTICLES)
        return fail(MITHRA_EINVAL, "%lld particles in the batch, at most %lld",
                    others + (long long)np, MAX_PARTICLES);
    mithra_status st = stage_particles(b.hs[sim], sim, np, pos, u, q_macro, m_macro);
    if (st) return st;
    b.committed = false;
    return MITHRA_OK;
}

mithra_status mithra_batch_config_diag(mithra_batch *bb, int32_t sim, const mithra_diag_cfg *cfg)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return config_diag(*bb->b, sim, cfg);
}

mithra_status mithra_batch_set_spectrum(mithra_batch *bb, int32_t sim, const double *nu,
                                        int32_t nfreq)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return set_spectrum(*bb->b, sim, nu, nfreq);
}

mithra_status mithra_batch_get_spectrum(mithra_batch *bb, int32_t sim, int64_t first_step,
                                        int64_t count, double *rest, double *lab)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return get_spectrum(*bb->b, sim, first_step, count, rest, lab);
}

mithra_status mithra_batch_set_seed(mithra_batch *bb, int32_t sim, const mithra_seed *seed)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return set_seed(*bb->b, sim, seed);
}

mithra_status mithra_batch_set_optical_undulator(mithra_batch *bb, int32_t sim,
                                                 const mithra_seed *wave)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return set_optical(*bb->b, sim, wave);
}

mithra_status mithra_batch_set_optical_beam(mithra_batch *bb, int32_t sim, const mithra_beam *beam)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return set_optical_beam(*bb->b, sim, beam);
}

mithra_status mithra_batch_set_seed_beam(mithra_batch *bb, int32_t sim, const mithra_beam *beam)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return set_seed_beam(*bb->b, sim, beam);
}

mithra_status mithra_batch_tune(mithra_batch *bb, int32_t trial_steps)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return tune(*bb->b, trial_steps);
}

mithra_status mithra_batch_set_shapes(mithra_batch *bb, const int32_t stencil_tile[3],
                                      const int32_t particle_brick[3])
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return set_shapes(*bb->b, stencil_tile, particle_brick);
}

mithra_status mithra_batch_run(mithra_batch *bb, int64_t nsteps)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return run(*bb->b, nsteps);
}

mithra_status mithra_batch_sync(mithra_batch *bb)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return sync(*bb->b);
}

mithra_status mithra_batch_get_diag(mithra_batch *bb, int32_t sim, mithra_diag_row *rows,
                                    int64_t cap, int64_t *nrows)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return get_diag(*bb->b, sim, rows, cap, nrows);
}

mithra_status mithra_batch_get_field(mithra_batch *bb, int32_t sim, mithra_field which, double *host)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return get_field(*bb->b, sim, which, host);
}

mithra_status mithra_batch_get_particles(mithra_batch *bb, int32_t sim, double *pos, double *u,
                                         uint8_t *alive, int64_t *np_alive)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return get_particles(*bb->b, sim, pos, u, alive, np_alive);
}

mithra_status mithra_batch_get_info(mithra_batch *bb, int32_t sim, mithra_info *info)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    return get_info(*bb->b, sim, info);
}

mithra_status mithra_batch_set_timing(mithra_batch *bb, int32_t on)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    bb->b->timing = on != 0;
    return MITHRA_OK;
}

mithra_status mithra_batch_get_timing(mithra_batch *bb, double *ms, int64_t *calls, int32_t nkinds,
                                      int32_t reset)
{
    if (!bb) return fail(MITHRA_EINVAL, "batch is NULL");
    mithra_sim tmp{bb->b};
    return mithra_get_timing(&tmp, ms, calls, nkinds, reset);
}

void mithra_batch_destroy(mithra_batch *bb)
{
    if (!bb) return;
    destroy_batch(bb->b);
    delete bb;
}

}  // extern "C"

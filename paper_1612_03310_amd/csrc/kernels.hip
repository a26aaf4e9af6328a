// gfx950 kernels of the boosted-frame FDTD/PIC step (arXiv:1612.03310,
// chapter "Methodology").  Every kernel serves a whole batch of independent
// simulations: a work table maps blocks to (simulation, tile).  The step
// counter lives in device memory, so one captured step replays unchanged.
//
// Nothing here is a dense contraction: every kernel is bound by HBM or LDS
// traffic, and none uses the matrix cores.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mithra_internal.hpp"

namespace mithra {

constexpr double C_LIGHT_D = 299792458.0;  // speed of light [m/s]

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Blocks are dispatched round-robin over the 8 XCDs of the chip, each with its
// own L2.  Remap so that every XCD gets a contiguous range of logical blocks:
// neighbouring tiles then share halo lines in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Particle work is concentrated where the bunch is.  The tiles are dealt to
// the XCDs in bricks of bs.x x bs.y x bs.z tiles: XCD x takes bricks x, x + 8,
// x + 16, ..., so every XCD gets a share of the dense region, while the tiles
// of a brick, which run at about the same time on one XCD, share their halo
// lines in its L2.  Inside a brick the tiles go x fastest.  The grid is
// padded to whole rounds of 8 bricks; a block past the last brick, or on a
// slot of an edge brick outside its simulation's grid, gets false.  sim and
// t: the simulation and its tile; g: the global tile index (tile0 + t).
__device__ __forceinline__ bool brick_tile(int b, const Brick *__restrict__ bricks, int nbricks,
                                           int4 bs, int &sim, int &t, int &g)
{
    const int x = b & 7, i = b >> 3;
    const int B = x + 8 * (i / bs.w), w = i % bs.w;
    if (B >= nbricks) return false;
    const Brick br = bricks[B];
    const int wx = w % bs.x, wy = (w / bs.x) % bs.y, wz = w / (bs.x * bs.y);
    const int tx = br.t0[0] + wx, ty = br.t0[1] + wy, tz = br.t0[2] + wz;
    if (tx >= br.nt[0] || ty >= br.nt[1] || tz >= br.nt[2]) return false;
    sim = br.sim;
    t = (tz * br.nt[1] + ty) * br.nt[0] + tx;
    g = br.g0 + (wz * br.nt[1] + wy) * br.nt[0] + wx;
    return true;
}

// index along an axis, wrapped on a periodic axis, clamped otherwise (clamped
// values are only ever read by points that do not use them).  The wrap is a
// full modulo: a stencil block wider than a periodic axis stages halo columns
// more than one period away, and every one of them must stay in the mesh.
__device__ __forceinline__ int axis_index(int v, int n, int periodic)
{
    if (v >= 0 && v < n) return v;
    if (!periodic) return v < 0 ? 0 : n - 1;
    const int r = v % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ void sin_cos(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void sin_cos(double x, double *s, double *c) { sincos(x, s, c); }

// seed signal shapes (section "FIELD", field-initialization), x = t - t0
__device__ double seed_signal(const SimDev &S, double t)
{
    const double x = t - S.seed_t0, ln2 = 0.69314718055994530942;
    const double carrier = cos(2.0 * 3.14159265358979323846 * S.seed_f * x + S.seed_cep);
    const double g = exp(-2.0 * ln2 * x * x / (S.seed_tau * S.seed_tau));
    switch (S.seed_sig) {
    case 0: return -S.seed_a0 * 4.0 * ln2 * carrier * x / (S.seed_tau * S.seed_tau) * g;
    case 1: return S.seed_a0 * carrier * g;
    case 2: return S.seed_a0 * carrier / cosh(x / S.seed_tau);
    default: return S.seed_a0 * carrier * (x <= 0.0 ? g : 1.0);
    }
}

// Envelope of the seed's signal at x = t - t0 (the signal is
// a0 e(x) cos(w x + cep)).
__device__ double seed_envelope(const SimDev &S, double x)
{
    const double ln2 = 0.69314718055994530942;
    const double g = exp(-2.0 * ln2 * x * x / (S.seed_tau * S.seed_tau));
    switch (S.seed_sig) {
    case 0: return -4.0 * ln2 * x / (S.seed_tau * S.seed_tau) * g;
    case 1: return g;
    case 2: return 1.0 / cosh(x / S.seed_tau);
    default: return x <= 0.0 ? g : 1.0;
    }
}

// Incident potential of a Gaussian-beam seed (travelling towards +z) for
// component comp at its grid point (i, j, k): A_x sits at x + dx/2, A_y at
// y + dy/2.  a0 p_c |U| e(x) cos(w x + cep + theta) with the paraxial
// envelope U = |U| exp(i theta) per axis v (xi along p/|p|, eta along
// z x p/|p|), zeta = z - z_f, m = zeta^2 + zr^2:
// |u| = (zr^2/m)^(1/4) exp(-k v^2 zr / (2m)), arg u = atan(zeta/zr)/2
// - k v^2 zeta / (2m).
__device__ double seed_beam_incident(const SimDev &S, int comp, int i, int j, int k, double t)
{
    const double x = S.origin[0] + ((double)i + (comp == 0 ? 0.5 : 0.0)) * S.d[0];
    const double y = S.origin[1] + ((double)j + (comp == 1 ? 0.5 : 0.0)) * S.d[1];
    const double z = S.origin[2] + (double)k * S.d[2];
    const double px = S.seed_p[0], py = S.seed_p[1], ipn = 1.0 / sqrt(px * px + py * py);
    const double X = x - S.seed_focus[0], Y = y - S.seed_focus[1], zeta = z - S.seed_focus[2];
    const double v[2] = {(X * px + Y * py) * ipn, (-X * py + Y * px) * ipn};
    double amp = 1.0, theta = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const double zr = S.seed_zr[a], im = 1.0 / (zeta * zeta + zr * zr);
        const double kv2 = S.seed_k * v[a] * v[a];
        amp *= sqrt(zr * sqrt(im)) * exp(-0.5 * kv2 * zr * im);
        theta += 0.5 * atan2(zeta, zr) - 0.5 * kv2 * zeta * im;
    }
    const double xs = t - (z - S.seed_zref) / C_LIGHT_D - S.seed_t0;
    const double w = 2.0 * 3.14159265358979323846 * S.seed_f;
    return S.seed_a0 * S.seed_p[comp] * amp * seed_envelope(S, xs) *
           cos(w * xs + S.seed_cep + theta);
}

// TF/SF corrections of a Gaussian-beam seed for one column and component:
// plane 2 (scattered side) loses what its update takes from the incident
// field on plane 3, plane 3 gains what its update misses on plane 2, each
// point with its own neighbours on the other plane (in the regrouped
// weights of the potential update: A (a_x, a_y) across, a_z along z).
__global__ __launch_bounds__(BLOCK) void k_seed_beam(const SimDev *__restrict__ sims, int sim,
                                                     int ncol, const long long *__restrict__ d_step)
{
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= 2 * ncol) return;
    const SimDev &S = sims[sim];
    const int comp = e / ncol, col = e - comp * ncol;
    const int i = col % S.n[0], j = col / S.n[0];
    const double t = (double)(*d_step) * S.dt;
    auto pull = [&](int k) {
        return S.A * (S.ax * (seed_beam_incident(S, comp, i + 1, j, k, t) +
                              seed_beam_incident(S, comp, i - 1, j, k, t)) +
                      S.ay * (seed_beam_incident(S, comp, i, j + 1, k, t) +
                              seed_beam_incident(S, comp, i, j - 1, k, t))) +
               S.az * seed_beam_incident(S, comp, i, j, k, t);
    };
    S.seed_corr[(long long)(2 * comp) * ncol + col] = -pull(3);
    S.seed_corr[(long long)(2 * comp + 1) * ncol + col] = pull(2);
}

// rho + background of one simulation, for the source of phi this step
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_background(const SimDev *__restrict__ sims, int sim,
                                                      long long ncell, Arena ar)
{
    const long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (c >= ncell) return;
    const SimDev &S = sims[sim];
    const R *rho = (const R *)ar.rho[*ar.d_step & 1] + S.cell0;
    ((R *)S.rho_bg)[c] = rho[c] + ((const R *)S.bg)[c];
}

// Rate ds/dt of the optical undulator's signal (the seed's four shapes with
// the undulator's parameters): carrier C = cos(w x + cep), envelope
// g = exp(-2 ln2 x^2 / tau^2), x = t - t0.
__device__ double optical_rate(const SimDev &S, double t)
{
    const double x = t - S.opt_t0, ln2 = 0.69314718055994530942;
    const double w = 2.0 * 3.14159265358979323846 * S.opt_f, it2 = 1.0 / (S.opt_tau * S.opt_tau);
    double sn, cs;
    sincos(w * x + S.opt_cep, &sn, &cs);
    const double g = exp(-2.0 * ln2 * x * x * it2);
    const double dg = -4.0 * ln2 * x * it2 * g;                 // g'
    switch (S.opt_sig) {
    case 0: {                                                   // a C g'
        const double ddg = -4.0 * ln2 * it2 * (g + x * dg);     // g''
        return S.opt_a * (cs * ddg - w * sn * dg);
    }
    case 1: return S.opt_a * (cs * dg - w * sn * g);            // a C g
    case 2: {                                                   // a C sech(x / tau)
        const double q = x / S.opt_tau, sech = 1.0 / cosh(q);
        return -S.opt_a * sech * (w * sn + cs * tanh(q) / S.opt_tau);
    }
    default:                                                    // Gaussian rise, then C
        return x <= 0.0 ? S.opt_a * (cs * dg - w * sn * g) : -S.opt_a * w * sn;
    }
}

// Envelope e and its rate e' of the optical undulator's signal at x = t - t0
// (the signal is a e(x) cos(w x + cep)).
__device__ void optical_envelope(const SimDev &S, double x, double *e, double *e1)
{
    const double ln2 = 0.69314718055994530942, it2 = 1.0 / (S.opt_tau * S.opt_tau);
    const double g = exp(-2.0 * ln2 * x * x * it2);
    const double dg = -4.0 * ln2 * x * it2 * g;
    switch (S.opt_sig) {
    case 0: *e = dg; *e1 = -4.0 * ln2 * it2 * (g + x * dg); break;
    case 1: *e = g; *e1 = dg; break;
    case 2: {
        const double q = x / S.opt_tau, sech = 1.0 / cosh(q);
        *e = sech;
        *e1 = -sech * tanh(q) / S.opt_tau;
        break;
    }
    default: *e = x <= 0.0 ? g : 1.0; *e1 = x <= 0.0 ? dg : 0.0; break;
    }
}

// Gaussian-beam optical undulator at (x, y, z, t): the plane wave's potential
// a p e(x) cos(phase) times the paraxial envelope U = |U| exp(i theta) of an
// astigmatic Gaussian beam travelling towards -z (per axis v = xi along p or
// eta along z x p with Rayleigh length zr, zeta = z_f - z, m = zeta^2 + zr^2:
// |u| = (zr^2/m)^(1/4) exp(-k v^2 zr / (2m)), arg u = atan(zeta/zr)/2
// - k v^2 zeta / (2m)).  With psi = a |U| e cos(Theta), Theta = w x + cep +
// theta, xi and eta along p/|p| and z x p/|p|: E = -p dpsi/dt,
// B = (-p_y, p_x) dpsi/dz and B_z = -|p| dpsi/deta, where
// the z and eta derivatives of U are U (alpha + i beta) with the real and
// imaginary parts written out below.
__device__ void optical_gaussian_beam(const SimDev &S, double t, double x, double y, double z,
                                      double *E, double *B)
{
    const double px = S.opt_p[0], py = S.opt_p[1], k = S.opt_k;
    const double pn = sqrt(px * px + py * py), ipn = 1.0 / pn;
    const double X = x - S.opt_focus[0], Y = y - S.opt_focus[1], zeta = S.opt_focus[2] - z;
    const double v[2] = {(X * px + Y * py) * ipn, (-X * py + Y * px) * ipn};
    double amp = 1.0, theta = 0.0, a_z = 0.0, b_z = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const double zr = S.opt_zr[a], m = zeta * zeta + zr * zr, im = 1.0 / m;
        const double kv2 = k * v[a] * v[a];
        amp *= sqrt(zr * sqrt(im)) * exp(-0.5 * kv2 * zr * im);
        theta += 0.5 * atan2(zeta, zr) - 0.5 * kv2 * zeta * im;
        a_z += -0.5 * zeta * im + kv2 * zeta * zr * im * im;
        b_z += 0.5 * zr * im + 0.5 * kv2 * (zeta * zeta - zr * zr) * im * im;
    }
    const double zr1 = S.opt_zr[1], im1 = 1.0 / (zeta * zeta + zr1 * zr1);
    const double a_eta = -k * v[1] * zr1 * im1, b_eta = -k * v[1] * zeta * im1;
    const double xs = t + (z - S.opt_zref) / C_LIGHT_D - S.opt_t0;
    const double w = 2.0 * 3.14159265358979323846 * S.opt_f;
    double e, e1, sn, cs;
    optical_envelope(S, xs, &e, &e1);
    sincos(w * xs + S.opt_cep + theta, &sn, &cs);
    const double aU = S.opt_a * amp;
    const double re = aU * e * cs, imv = aU * e * sn;   // a Re{U S}, a Im{U S}
    const double dt_psi = aU * (e1 * cs - w * e * sn);  // a Re{U S'}
    const double dz_psi = dt_psi / C_LIGHT_D - (a_z * re - b_z * imv);
    const double deta_psi = a_eta * re - b_eta * imv;
    E[0] = -px * dt_psi;
    E[1] = -py * dt_psi;
    B[0] = -py * dz_psi;
    B[1] = px * dz_psi;
    B[2] = -pn * deta_psi;
}

__device__ __forceinline__ int comp_extent(const SimDev &S, int c, int a)
{
    return (c == a && !S.bc[a]) ? S.n[a] - 1 : S.n[a];
}

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive scan over a 256-thread block; returns the prefix, total in *tot
__device__ __forceinline__ int block_excl_scan(int v, int *sh /*[4]*/, int *tot)
{
    const int incl = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) sh[w] = incl;
    __syncthreads();
    int base = 0, all = 0;
#pragma unroll
    for (int i = 0; i < BLOCK / 64; ++i) {
        const int s = sh[i];
        if (i < w) base += s;
        all += s;
    }
    __syncthreads();
    *tot = all;
    return base + incl - v;
}

// fixed-order tree reduction of one double per thread over a 256-thread block
__device__ __forceinline__ double block_sum(double v, double *sh /*[256]*/)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// vertex fields (section "Field Evaluation"): E and B at vertex (i, j, k) at
// t_{s+1/2} from A^s, A^{s+1} and phi^s; the vertex value of the edge-sampled
// A_l is the mean of its two edges along l.  B is the mean of the central
// curls at the two levels; the sum over levels is taken first.
// ---------------------------------------------------------------------------

template <typename R>
struct FieldPtrs {
    const R *A0[3];
    const R *A1[3];
    const R *phi;
};

template <typename R>
__device__ __forceinline__ FieldPtrs<R> field_ptrs(const SimDev &S, const Arena &ar,
                                                   long long lev0, long long lev1, int phi_lev)
{
    FieldPtrs<R> f;
    for (int c = 0; c < 3; ++c) {
        f.A0[c] = (const R *)ar.pot[lev0][c] + S.cell0;
        f.A1[c] = (const R *)ar.pot[lev1][c] + S.cell0;
    }
    f.phi = (const R *)ar.pot[phi_lev][3] + S.cell0;
    return f;
}

template <typename R>
__device__ __forceinline__ void vertex_EB(const SimDev &S, const FieldPtrs<R> &f, int i, int j,
                                          int k, R E[3], R B[3])
{
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const long long sy = nx, sz = (long long)nx * ny;
    const int im = axis_index(i - 1, nx, S.bc[0]), ip = axis_index(i + 1, nx, S.bc[0]);
    const int jm = axis_index(j - 1, ny, S.bc[1]), jp = axis_index(j + 1, ny, S.bc[1]);
    const int km = axis_index(k - 1, nz, S.bc[2]), kp = axis_index(k + 1, nz, S.bc[2]);
    auto at = [&](int a, int b, int c) { return (long long)c * sz + (long long)b * sy + a; };
    const R h = (R)0.5, q = (R)0.25;
    const R idt = (R)S.inv_dt, i2x = (R)S.inv_2d[0], i2y = (R)S.inv_2d[1], i2z = (R)S.inv_2d[2];
    const R *ph = f.phi;
    // E = -dA/dt - grad phi
    {
        const long long p = at(i, j, k), px = at(im, j, k), py = at(i, jm, k), pz = at(i, j, km);
        const R dAx = h * ((f.A1[0][p] + f.A1[0][px]) - (f.A0[0][p] + f.A0[0][px]));
        const R dAy = h * ((f.A1[1][p] + f.A1[1][py]) - (f.A0[1][p] + f.A0[1][py]));
        const R dAz = h * ((f.A1[2][p] + f.A1[2][pz]) - (f.A0[2][p] + f.A0[2][pz]));
        E[0] = -dAx * idt - (ph[at(ip, j, k)] - ph[at(im, j, k)]) * i2x;
        E[1] = -dAy * idt - (ph[at(i, jp, k)] - ph[at(i, jm, k)]) * i2y;
        E[2] = -dAz * idt - (ph[at(i, j, kp)] - ph[at(i, j, km)]) * i2z;
    }
    // level sums of A at an edge sample
    auto S0 = [&](int c, long long p) { return f.A0[c][p] + f.A1[c][p]; };
    // Bx = dAz/dy - dAy/dz
    {
        const R dz_dy = (S0(2, at(i, jp, k)) + S0(2, at(i, jp, km))) -
                        (S0(2, at(i, jm, k)) + S0(2, at(i, jm, km)));
        const R dy_dz = (S0(1, at(i, j, kp)) + S0(1, at(i, jm, kp))) -
                        (S0(1, at(i, j, km)) + S0(1, at(i, jm, km)));
        B[0] = q * (dz_dy * i2y - dy_dz * i2z);
    }
    // By = dAx/dz - dAz/dx
    {
        const R dx_dz = (S0(0, at(i, j, kp)) + S0(0, at(im, j, kp))) -
                        (S0(0, at(i, j, km)) + S0(0, at(im, j, km)));
        const R dz_dx = (S0(2, at(ip, j, k)) + S0(2, at(ip, j, km))) -
                        (S0(2, at(im, j, k)) + S0(2, at(im, j, km)));
        B[1] = q * (dx_dz * i2z - dz_dx * i2x);
    }
    // Bz = dAy/dx - dAx/dy
    {
        const R dy_dx = (S0(1, at(ip, j, k)) + S0(1, at(ip, jm, k))) -
                        (S0(1, at(im, j, k)) + S0(1, at(im, jm, k)));
        const R dx_dy = (S0(0, at(i, jp, k)) + S0(0, at(im, jp, k))) -
                        (S0(0, at(i, jm, k)) + S0(0, at(im, jm, k)));
        B[2] = q * (dy_dx * i2x - dx_dy * i2y);
    }
}

// vertices where the E, B formulas are evaluated: [1, n-2] on a Mur axis
__device__ __forceinline__ bool vertex_valid(const SimDev &S, int i, int j, int k)
{
    const int v[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (v[a] < 0 || v[a] >= S.n[a]) return false;
        if (!S.bc[a] && (v[a] < 1 || v[a] > S.n[a] - 2)) return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// 1. potential update, eq. (updateEquation), all four components.
//    Each thread owns an (x, y) column and marches z through a block's chunk
//    of planes.  Plane k+1 of psi^s is staged with a one-cell halo in a
//    three-slot LDS ring (one barrier per plane: each iteration reads only the
//    plane it staged, older planes stay in registers); loads run one plane
//    ahead through registers so that a block keeps two planes in flight.  With
//      T_k = ax (P_{i+1} + P_{i-1}) + ay (P_{j+1} + P_{j-1}) at plane k,
//    the update is
//      psi^{s+1} = -psi^{s-1} + a1 P + A (T_{k-1} + T_{k+1}) + (1 - 2A) T_k
//                  + az (P_{k+1} + P_{k-1}) + src S,
//    an exact regrouping of the z-averaged transverse neighbours.
//    With fuse_x the same pass applies Mur on the two x faces (points with y
//    and z inside; the boundary kernels keep the y and z faces, edges and
//    corners): the face's inward neighbour along x is the adjacent lane of
//    the wavefront, whose psi^{s-1}, psi^s and fresh psi^{s+1} arrive by
//    shuffle; for second order the transverse neighbours at level s come
//    from the plane-k LDS slot (y) and the z-march registers (z).
//    The host enables it only when no face column sits at a wavefront edge.
// ---------------------------------------------------------------------------

template <typename R, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void k_stencil(const SimDev *__restrict__ sims,
                                                     const int4 *__restrict__ items, Arena ar,
                                                     int KZ, int fuse_x)
{
    const int4 it = items[xcd_remap(blockIdx.x, gridDim.x)];
    const SimDev &S = sims[it.x];
    const int comp = blockIdx.y;
    if (comp == 3 && !S.sc) return;
    const long long step = *ar.d_step;
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const long long sxy = (long long)nx * ny;
    const R *__restrict__ P = (const R *)ar.pot[step % 3][comp] + S.cell0;
    const R *__restrict__ Q = (const R *)ar.pot[(step + 2) % 3][comp] + S.cell0;
    R *__restrict__ Rn = (R *)ar.pot[(step + 1) % 3][comp] + S.cell0;
    // with a static background charge, phi's source is rho + background
    const R *__restrict__ Src =
        comp < 3 ? (const R *)ar.J[comp] + S.cell0
                 : (S.rho_bg ? (const R *)S.rho_bg : (const R *)ar.rho[step & 1] + S.cell0);

    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = S.bc[a] ? 0 : 1;
        hi[a] = S.bc[a] ? S.n[a] - 1 : comp_extent(S, comp, a) - 2;
    }
    const int k0 = max(it.w * KZ, lo[2]);
    const int k1 = min(it.w * KZ + KZ - 1, hi[2]);
    if (k0 > k1) return;  // uniform over the block

    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int i = it.y * TX + tx, j = it.z * TY + ty;
    const bool act = i >= lo[0] && i <= hi[0] && j >= lo[1] && j <= hi[1];
    const int ext0 = comp_extent(S, comp, 0);
    const bool face = fuse_x && !S.bc[0] && j >= lo[1] && j <= hi[1] && (i == 0 || i == ext0 - 1);
    const bool m2 = S.mur2 != 0;
    // first order: beta_0, beta_1; second order: gamma_0, gamma_1, and the
    // transverse weights along y and z
    const R mb0 = (R)(m2 ? S.murg[0][0] : S.murb0[0]), mb1 = (R)(m2 ? S.murg[0][1] : S.murb1[0]);
    const R mgy = (R)S.murg[0][2], mgz = (R)S.murg[0][3];
    // seed plane wave (total-field/scattered-field): the scattered-field plane
    // k = 2 loses what its update took from the incident field on plane 3,
    // which gains what its update missed on plane 2; both corrections are
    // uniform over the plane
    const bool seeded = S.seed_on && comp < 2 && S.seed_p[comp < 2 ? comp : 0] != 0.0 && !S.bc[2];
    R corr_s = 0, corr_t = 0;
    if (seeded && S.seed_beam) {
        // a Gaussian beam: per-column corrections written before this launch
        if (act && k0 <= 3) {
            const long long cc = (long long)j * nx + i;
            corr_s = (R)S.seed_corr[(2 * comp) * sxy + cc];
            corr_t = (R)S.seed_corr[(2 * comp + 1) * sxy + cc];
        }
    } else if (seeded) {
        const double t = (double)step * S.dt;
        const double wgt = S.A * (2.0 * S.ax + 2.0 * S.ay) + S.az;  // weight of plane k +- 1
        const double p = S.seed_p[comp];
        corr_s = (R)(-wgt * p * seed_signal(S, t - (S.origin[2] + 3.0 * S.d[2] - S.seed_zref) / C_LIGHT_D));
        corr_t = (R)(wgt * p * seed_signal(S, t - (S.origin[2] + 2.0 * S.d[2] - S.seed_zref) / C_LIGHT_D));
    }

    const R a1 = (R)S.a1, ax = (R)S.ax, ay = (R)S.ay, az = (R)S.az, A = (R)S.A;
    const R oma = (R)(1.0 - 2.0 * S.A);
    const R src = (R)(comp < 3 ? S.srcA : S.srcPhi);

    __shared__ R sP[3][TY + 2][TX + 2];
    // each thread stages at most NE elements of a haloed plane; their plane
    // offsets do not depend on k
    constexpr int NT = TX * TY, NPL = (TX + 2) * (TY + 2), NE = (NPL + NT - 1) / NT;
    int eoff[NE], elds[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        const int e = threadIdx.x + m * NT;
        const int lx = e % (TX + 2), ly = e / (TX + 2);
        const int gi = axis_index(it.y * TX - 1 + lx, nx, S.bc[0]);
        const int gj = axis_index(it.z * TY - 1 + ly, ny, S.bc[1]);
        eoff[m] = gj * nx + gi;
        elds[m] = e < NPL ? e : -1;
    }
    R pv[NE];
    auto fetch = [&](int kk) {  // global -> registers
        const R *base = P + (long long)axis_index(kk, nz, S.bc[2]) * sxy;
#pragma unroll
        for (int m = 0; m < NE; ++m)
            if (elds[m] >= 0) pv[m] = base[eoff[m]];
    };
    auto commit = [&](int slot) {  // registers -> LDS
#pragma unroll
        for (int m = 0; m < NE; ++m)
            if (elds[m] >= 0) (&sP[slot][0][0])[elds[m]] = pv[m];
    };
    auto trans = [&](int slot) {
        return ax * (sP[slot][ty + 1][tx + 2] + sP[slot][ty + 1][tx]) +
               ay * (sP[slot][ty + 2][tx + 1] + sP[slot][ty][tx + 1]);
    };

    // software pipeline: while plane k is computed, plane k+2 of psi^s and
    // psi^{s-1}, S at plane k+1 are already in flight
    const long long col = (long long)j * nx + i;
    fetch(k0 - 1);
    commit(0);
    fetch(k0);
    commit(1);
    fetch(k0 + 1);
    R qn = 0, sn = 0;
    if (act || face) qn = __builtin_nontemporal_load(&Q[(long long)k0 * sxy + col]);
    if (act) sn = __builtin_nontemporal_load(&Src[(long long)k0 * sxy + col]);
    __syncthreads();
    R Tm = trans(0), Tc = trans(1);
    R Pm = sP[0][ty + 1][tx + 1], Pc = sP[1][ty + 1][tx + 1];
    int slot = 2;
    for (int k = k0; k <= k1; ++k) {
        // the slot refilled here was last read two iterations ago, before the
        // previous barrier
        commit(slot);
        const R q = qn, s = sn;
        if (k < k1) {
            fetch(k + 2);
            if (act || face) qn = __builtin_nontemporal_load(&Q[(long long)(k + 1) * sxy + col]);
            if (act) sn = __builtin_nontemporal_load(&Src[(long long)(k + 1) * sxy + col]);
        }
        __syncthreads();
        const R Pp = sP[slot][ty + 1][tx + 1];
        const R Tp = trans(slot);
        R val = -q + a1 * Pc + A * (Tm + Tp) + oma * Tc + az * (Pp + Pm) + src * s;
        if (seeded) val += k == 2 ? corr_s : (k == 3 ? corr_t : (R)0);
        if (act) __builtin_nontemporal_store(val, &Rn[(long long)k * sxy + col]);
        if (fuse_x) {
            // the low face reads lane + 1, the high face lane - 1
            const R vd = __shfl_down(val, 1), qd = __shfl_down(q, 1), pd = __shfl_down(Pc, 1);
            const R vu = __shfl_up(val, 1), qu = __shfl_up(q, 1), pu = __shfl_up(Pc, 1);
            R trv = 0;  // second order: transverse neighbours at level s, both layers
            if (m2) {
                const R pmd = __shfl_down(Pm, 1), ppd = __shfl_down(Pp, 1);
                const R pmu = __shfl_up(Pm, 1), ppu = __shfl_up(Pp, 1);
                if (face) {
                    const bool low = i == 0;
                    // plane k sits in the slot before the one plane k+1 just went to
                    const int cs = slot == 0 ? 2 : slot - 1;
                    const int xi = low ? tx + 2 : tx;                     // the inner column
                    trv = mgy * ((sP[cs][ty + 2][tx + 1] + sP[cs][ty][tx + 1]) +
                                 (sP[cs][ty + 2][xi] + sP[cs][ty][xi])) +
                          mgz * ((Pp + Pm) + (low ? ppd + pmd : ppu + pmu));
                }
            }
            if (face) {
                const bool low = i == 0;
                const R vq = low ? vd : vu, Qq = low ? qd : qu, Pq = low ? pd : pu;
                __builtin_nontemporal_store(mb0 * q + mb1 * Pc - Qq + mb1 * Pq + mb0 * vq + trv,
                                            &Rn[(long long)k * sxy + col]);
            }
        }
        Pm = Pc;
        Pc = Pp;
        Tm = Tc;
        Tc = Tp;
        slot = slot == 2 ? 0 : slot + 1;
    }
}

// ---------------------------------------------------------------------------
// 2. first-order Mur on the outer layer of every component grid (section
//    "Boundary Truncation").  A point on several faces uses the rule of its
//    highest-priority axis (z > y > x); its inward neighbour along that axis
//    lies on one face fewer.  Each thread evaluates that chain down to an
//    interior point, so faces, edges and corners need no ordering between
//    threads: only interior psi^{s+1} values are read.
// ---------------------------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_boundary(const SimDev *__restrict__ sims,
                                                     const BSeg *__restrict__ segs, int nseg,
                                                     long long total, Arena ar)
{
    const long long step = *ar.d_step;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < total;
         t += (long long)gridDim.x * BLOCK) {
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segs[mid].start <= t) lo = mid;
            else hi = mid - 1;
        }
        const BSeg g = segs[lo];
        const SimDev &S = sims[g.sim];
        const int c = g.comp;
        const long long r = t - g.start;
        int ext[3], ilo[3], ihi[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ext[a] = comp_extent(S, c, a);
            ilo[a] = S.bc[a] ? 0 : 1;
            ihi[a] = S.bc[a] ? ext[a] - 1 : ext[a] - 2;
        }
        int v[3];
        if (g.group == 2) {
            const long long fa = (long long)ext[0] * ext[1];
            const int face = (int)(r / fa), rem = (int)(r % fa);
            v[0] = rem % ext[0];
            v[1] = rem / ext[0];
            v[2] = face ? ext[2] - 1 : 0;
        } else if (g.group == 1) {
            const int nzi = ihi[2] - ilo[2] + 1;
            const long long fa = (long long)ext[0] * nzi;
            const int face = (int)(r / fa), rem = (int)(r % fa);
            v[0] = rem % ext[0];
            v[2] = ilo[2] + rem / ext[0];
            v[1] = face ? ext[1] - 1 : 0;
        } else {
            const int nyi = ihi[1] - ilo[1] + 1, nzi = ihi[2] - ilo[2] + 1;
            const long long fa = (long long)nyi * nzi;
            const int face = (int)(r / fa), rem = (int)(r % fa);
            v[1] = ilo[1] + rem % nyi;
            v[2] = ilo[2] + rem / nyi;
            v[0] = face ? ext[0] - 1 : 0;
        }
        const R *P = (const R *)ar.pot[step % 3][c] + S.cell0;
        const R *Q = (const R *)ar.pot[(step + 2) % 3][c] + S.cell0;
        R *Rn = (R *)ar.pot[(step + 1) % 3][c] + S.cell0;
        const long long sy = S.n[0], sz = (long long)S.n[0] * S.n[1];
        long long pts[4];
        int axs[3];
        int len = 0;
        int cur[3] = {v[0], v[1], v[2]};
        for (;;) {
            int top = -1;
            for (int a = 2; a >= 0; --a)
                if (!S.bc[a] && (cur[a] == 0 || cur[a] == ext[a] - 1)) {
                    top = a;
                    break;
                }
            if (top < 0) break;
            pts[len] = cur[2] * sz + cur[1] * sy + cur[0];
            axs[len] = top;
            ++len;
            cur[top] += cur[top] == 0 ? 1 : -1;
        }
        pts[len] = cur[2] * sz + cur[1] * sy + cur[0];
        R val = Rn[pts[len]];
        for (int m = len - 1; m >= 0; --m) {
            const R b0 = (R)S.murb0[axs[m]], b1 = (R)S.murb1[axs[m]];
            const long long p = pts[m], q = pts[m + 1];
            val = b0 * Q[p] + b1 * P[p] - Q[q] + b1 * P[q] + b0 * val;
        }
        Rn[pts[0]] = val;
    }
}

// ---------------------------------------------------------------------------
// 2b. second-order Mur (section "Boundary Truncation"), in three launches:
//     faces (points on one face), then edges, then corners, each reading
//     only psi^{s+1} values written before it.  On a face normal to a, with
//     b the boundary point, q its inward neighbour and u, w the other axes:
//       psi^{s+1}_b = g0 (psi^{s-1}_b + psi^{s+1}_q) + g1 (psi^s_b + psi^s_q)
//                     - psi^{s-1}_q + gu sum_{+-u} (psi^s_b + psi^s_q)
//                     + gw sum_{+-w} (psi^s_b + psi^s_q)
//     (the printed gamma coefficients).  Edges and corners: the face
//     conditions involved, added in inward coordinates and discretised at
//     the centre of the edge square or corner cube, with the second
//     derivatives along the face normals replaced through the wave
//     equation:  (d_sa + d_sb) d_t - 3/(2c) d_tt + c/2 d_ee = 0 on an edge
//     along e, (d_sa + d_sb + d_sc) d_t - 2/c d_tt = 0 at a corner; each is
//     solved for the one unknown corner of the square or cube.
// ---------------------------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_mur2(const SimDev *__restrict__ sims,
                                                 const BSeg *__restrict__ segs, int nseg,
                                                 long long total, Arena ar)
{
    const long long step = *ar.d_step;
    for (long long t = (long long)blockIdx.x * BLOCK + threadIdx.x; t < total;
         t += (long long)gridDim.x * BLOCK) {
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segs[mid].start <= t) lo = mid;
            else hi = mid - 1;
        }
        const BSeg g = segs[lo];
        const SimDev &S = sims[g.sim];
        const int c = g.comp;
        const long long r = t - g.start;
        int ext[3], ilo[3], nin[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ext[a] = comp_extent(S, c, a);
            ilo[a] = S.bc[a] ? 0 : 1;
            nin[a] = S.bc[a] ? ext[a] : ext[a] - 2;
        }
        const R *P = (const R *)ar.pot[step % 3][c] + S.cell0;
        const R *Q = (const R *)ar.pot[(step + 2) % 3][c] + S.cell0;
        R *Rn = (R *)ar.pot[(step + 1) % 3][c] + S.cell0;
        auto idx = [&](const int *v) {
            const int i = axis_index(v[0], S.n[0], S.bc[0]);
            const int j = axis_index(v[1], S.n[1], S.bc[1]);
            const int k = axis_index(v[2], S.n[2], S.bc[2]);
            return ((long long)k * S.n[1] + j) * S.n[0] + i;
        };
        int v[3];
        if (g.group < 3) {
            const int a = g.group, u = a == 0 ? 1 : 0, w = a == 2 ? 1 : 2;
            const long long fa = (long long)nin[u] * nin[w];
            const int side = (int)(r / fa), rem = (int)(r % fa);
            v[u] = ilo[u] + rem % nin[u];
            v[w] = ilo[w] + rem / nin[u];
            v[a] = side ? ext[a] - 1 : 0;
            int q[3] = {v[0], v[1], v[2]};
            q[a] += side ? -1 : 1;
            double tr = 0.0;
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const int ax = tt ? w : u;
                const double gt = S.murg[a][2 + tt];
#pragma unroll
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    int vb[3] = {v[0], v[1], v[2]}, vq[3] = {q[0], q[1], q[2]};
                    vb[ax] += sgn;
                    vq[ax] += sgn;
                    tr += gt * ((double)P[idx(vb)] + (double)P[idx(vq)]);
                }
            }
            const long long pb = idx(v), pq = idx(q);
            const double g0 = S.murg[a][0], g1 = S.murg[a][1];
            Rn[pb] = (R)(g0 * ((double)Q[pb] + (double)Rn[pq]) + g1 * ((double)P[pb] + (double)P[pq]) -
                         (double)Q[pq] + tr);
        } else if (g.group < 6) {
            const int e = g.group - 3, a = e == 0 ? 1 : 0, b = e == 2 ? 1 : 2;
            const int corner = (int)(r / nin[e]);
            v[e] = ilo[e] + (int)(r % nin[e]);
            const int sa = corner & 1, sb = corner >> 1;
            v[a] = sa ? ext[a] - 1 : 0;
            v[b] = sb ? ext[b] - 1 : 0;
            // square points (ia, ib): ia, ib = steps inward along a, b
            double Rv[2][2], Pv[2][2], Qv[2][2], De = 0.0;
#pragma unroll
            for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                for (int ia = 0; ia < 2; ++ia) {
                    int pt[3] = {v[0], v[1], v[2]};
                    pt[a] += ia * (sa ? -1 : 1);
                    pt[b] += ib * (sb ? -1 : 1);
                    const long long p = idx(pt);
                    Rv[ia][ib] = (ia | ib) ? (double)Rn[p] : 0.0;
                    Pv[ia][ib] = (double)P[p];
                    Qv[ia][ib] = (double)Q[p];
                    int pp[3] = {pt[0], pt[1], pt[2]}, pm[3] = {pt[0], pt[1], pt[2]};
                    pp[e] += 1;
                    pm[e] -= 1;
                    De += (double)P[idx(pp)] - 2.0 * Pv[ia][ib] + (double)P[idx(pm)];
                }
            const double ka = 0.25 / (S.dt * S.d[a]), kb = 0.25 / (S.dt * S.d[b]);
            const double kt = 3.0 / (8.0 * C_LIGHT_D * S.dt * S.dt);
            const double ke = C_LIGHT_D / (8.0 * S.d[e] * S.d[e]);
            double sP = 0.0, sQ = 0.0;
#pragma unroll
            for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                for (int ia = 0; ia < 2; ++ia) {
                    sP += Pv[ia][ib];
                    sQ += Qv[ia][ib];
                }
            const double rest =
                ka * ((Rv[1][0] - Qv[1][0] + Qv[0][0]) + (Rv[1][1] - Rv[0][1]) - (Qv[1][1] - Qv[0][1])) +
                kb * ((Rv[0][1] - Qv[0][1] + Qv[0][0]) + (Rv[1][1] - Rv[1][0]) - (Qv[1][1] - Qv[1][0])) -
                kt * ((Rv[1][0] + Rv[0][1] + Rv[1][1]) - 2.0 * sP + sQ) + ke * De;
            Rn[idx(v)] = (R)(rest / (ka + kb + kt));
        } else {
            const int corner = (int)r;
            int sd[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                sd[a] = (corner >> a) & 1;
                v[a] = sd[a] ? ext[a] - 1 : 0;
            }
            double k[3], kt = 1.0 / (4.0 * C_LIGHT_D * S.dt * S.dt), rest = 0.0, den = kt;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                k[a] = 0.125 / (S.dt * S.d[a]);
                den += k[a];
            }
            double sR = 0.0, sP = 0.0, sQ = 0.0;
            for (int m = 0; m < 8; ++m) {
                int pt[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) pt[a] = v[a] + ((m >> a) & 1) * (sd[a] ? -1 : 1);
                const long long p = idx(pt);
                const double rv = m ? (double)Rn[p] : 0.0, qv = (double)Q[p];
                sR += rv;
                sP += (double)P[p];
                sQ += qv;
                // d_s d_t along each axis: inner layer minus outer layer
#pragma unroll
                for (int a = 0; a < 3; ++a) rest += k[a] * (((m >> a) & 1) ? 1.0 : -1.0) * (rv - qv);
            }
            rest -= kt * (sR - 2.0 * sP + sQ);
            Rn[idx(v)] = (R)(rest / den);
        }
    }
}

// ---------------------------------------------------------------------------
// 3. gather + undulator + Boris push, one block per 8^3-cell tile.
//    The tile's particles are contiguous (sorted by cell at the end of the
//    previous step).  E and B at the tile's 9^3 vertices are computed once
//    into LDS (pre-scaled to Boris kicks), then every particle interpolates
//    linearly (eq. (fieldInterpolation)), adds the rest-frame undulator field
//    at each sub-step, and is pushed (eq. (BorisScheme)).  Positions are kept
//    as an int32 cell (the bin key) plus an offset in [0, 1) per axis.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int tile_key(const SimDev &S, int ci, int cj, int ck)
{
    const int t = ((ck >> 3) * S.nt[1] + (cj >> 3)) * S.nt[0] + (ci >> 3);
    return t * TILE_CELLS + (((ck & 7) * TILE + (cj & 7)) * TILE + (ci & 7));
}

// rest-frame undulator field (eqs. (undulatorField), (undulatorFieldRest) with
// E_x = -g0 b0 c B'_y, and the fringe field for z' < 0), scaled to kicks.
// ph_cell: k_u z' at the particle's cell corner, in double (it reaches
// hundreds of radians); the in-cell part is added in working precision.
template <typename R>
__device__ __forceinline__ void undulator_kick(const SimDev &S, double ph_cell, R fz, double y,
                                               R &Ex, R &By, R &Bz)
{
    const double kzc = S.kz_cell;
    const double full = ph_cell + kzc * (double)fz;
    const R kuy = (R)(S.ku * y);
    const R ch = cosh(kuy), sh = sinh(kuy);
    if (S.und_kL > 0.0 && full > S.und_kL) {
        // past the exit of a finite undulator: the entrance fringe mirrored
        // about z' = L
        const R s = (R)((ph_cell - S.und_kL) + kzc * (double)fz);
        const R g = exp(-s * s * (R)0.5);
        Ex = (R)S.EuK * ch * s * g;
        By = (R)S.BuyK * ch * s * g;
        Bz = (R)S.BuzK * sh * g;
    } else if (full >= 0.0) {
        const double twopi = 6.283185307179586476925286766559;
        const double red = ph_cell - twopi * floor(ph_cell / twopi);
        const R ph = (R)red + (R)kzc * fz;
        R sn, cs;
        sin_cos(ph, &sn, &cs);
        Ex = (R)S.EuK * ch * sn;
        By = (R)S.BuyK * ch * sn;
        Bz = (R)S.BuzK * sh * cs;
    } else {
        const R s = (R)full;
        const R g = exp(-s * s * (R)0.5);
        Ex = (R)S.EuK * ch * s * g;
        By = (R)S.BuyK * ch * s * g;
        Bz = (R)S.BuzK * sh * g;
    }
}

// One atomic add per run of equal keys in consecutive active lanes of a
// wavefront (particles arrive sorted by cell, so runs are common).  Every lane
// of the wavefront must call this.
__device__ __forceinline__ void count_runs(int *counts, int key, bool active)
{
    const int lane = threadIdx.x & 63;
    const int k = active ? key : -1;
    const int prev = __shfl_up(k, 1, 64);
    const bool head = active && (lane == 0 || prev != k);
    const unsigned long long heads = __ballot(head);
    const unsigned long long act = __ballot(active);
    if (head) {
        const unsigned long long later = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
        const int next = later ? __ffsll((long long)later) - 1 : 64;
        const unsigned long long span =
            (next == 64 ? ~0ull : ((1ull << next) - 1)) & (~0ull << lane);
        atomicAdd(&counts[k], __popcll(act & span));
    }
}

// OPTICAL: the variant that also evaluates the optical undulator (its FP64
// transcendentals would otherwise raise the register count of every launch).
// The single-precision kernel is held to 80 registers, six waves per SIMD:
// the push gains from every tile in flight on a compute unit (it contends
// for the vector-memory pipeline), and 80 is what it needs without spilling
// once no particle is held in registers while the field table is built.
template <typename R, bool OPTICAL>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(OPTICAL ? 1 : sizeof(R) == 4 ? 6 : 1))) void k_push(
    const SimDev *__restrict__ sims, const Brick *__restrict__ bricks, int nbricks, int4 bs,
    Arena ar)
{
    int sim, tl, ti;  // ti: the global tile index
    if (!brick_tile(blockIdx.x, bricks, nbricks, bs, sim, tl, ti)) return;
    // A tile that no particle entered in the previous step (flag written by
    // that step's push, or set for all tiles after particles are loaded) has
    // nothing to do: one round trip decides it.
    const int occ0 = ar.pocc[0][ti], occ1 = ar.pocc[1][ti];
    const long long step = *ar.d_step;
    const int par = (int)(step & 1);
    if ((par ? occ1 : occ0) == 0) return;
    const int2 it = make_int2(sim, tl);
    const SimDev &S = sims[it.x];
    const int *__restrict__ offs = ar.offs[par];
    if (it.y == 0 && threadIdx.x == 0) {
        // particles lost in earlier steps stay in the lost bucket; tile 0
        // runs every step for that
        const long long g = S.key0 + S.nkeys;
        const int n_lost = offs[g + 1] - offs[g];
        if (n_lost) atomicAdd(&ar.counts[g], n_lost);
        ar.pocc[par ^ 1][ti] = 1;
    }
    const long long g0 = S.key0 + (long long)it.y * TILE_CELLS;
    const int p_lo = offs[g0], p_hi = offs[g0 + TILE_CELLS];
    if (p_lo == p_hi) {
        if (threadIdx.x == 0 && it.y != 0) ar.pocc[par][ti] = 0;
        return;
    }

    const int t = it.y;
    const int L0 = (t % S.nt[0]) * TILE, L1 = ((t / S.nt[0]) % S.nt[1]) * TILE,
              L2 = (t / (S.nt[0] * S.nt[1])) * TILE;
    if (threadIdx.x < 27) {
        // the deposit of the tiles around this one has work
        const int a = L0 / TILE + (int)threadIdx.x % 3 - 1,
                  b = L1 / TILE + ((int)threadIdx.x / 3) % 3 - 1,
                  cc = L2 / TILE + (int)threadIdx.x / 9 - 1;
        if (a >= 0 && a < S.nt[0] && b >= 0 && b < S.nt[1] && cc >= 0 && cc < S.nt[2])
            ar.tact[S.tile0 + (cc * S.nt[1] + b) * S.nt[0] + a] = 1;
    }

    int *__restrict__ key = ar.key[par];
    R *__restrict__ o0 = (R *)ar.off[par][0];
    R *__restrict__ o1 = (R *)ar.off[par][1];
    R *__restrict__ o2 = (R *)ar.off[par][2];
    R *__restrict__ u0 = (R *)ar.u[par][0];
    R *__restrict__ u1 = (R *)ar.u[par][1];
    R *__restrict__ u2 = (R *)ar.u[par][2];

    // The particle's key, offset and momentum.  In the single-precision
    // kernel they are loaded in the particle loop, after the field table:
    // held across the table they would cost the registers of a sixth wave.
    // The double-precision kernel (held by its LDS to three blocks per
    // compute unit) and the optical one (by its registers to two waves) lose
    // no wave by holding them: there the thread's first particle is loaded
    // with the potentials, so that the block waits for memory once.
    constexpr bool PRELOAD = sizeof(R) == 8 || OPTICAL;
    int gk = 0;
    R f[3] = {0, 0, 0}, u[3] = {0, 0, 0};
    if (PRELOAD && p_lo + (int)threadIdx.x < p_hi) {
        const int p = p_lo + threadIdx.x;
        gk = key[p];
        f[0] = o0[p];
        f[1] = o1[p];
        f[2] = o2[p];
        u[0] = u0[p];
        u[1] = u1[p];
        u[2] = u2[p];
    }

    // E and B at the tile's 9^3 vertices, from the potentials of the box
    // [L-1, L+9]^3 in two passes over one LDS staging area of 4 x 11^3
    // values: first the level differences of A (for E = -dA/dt) and phi,
    // then the level sums of A (for B, the mean of curl A over the two
    // levels).  E waits in registers during the second pass; the kick-scaled
    // table then overwrites the staging.
    constexpr int NV = TILE_VERT * TILE_VERT * TILE_VERT;  // 729
    constexpr int SG = TILE_VERT + 2;                      // 11
    constexpr int NS = SG * SG * SG;                       // 1331
    constexpr int NSE = (NS + BLOCK - 1) / BLOCK;          // staged points per thread
    constexpr int VPT = (NV + BLOCK - 1) / BLOCK;          // vertices per thread
    constexpr int OX = 1, OY = SG, OZ = SG * SG;
    static_assert(6 * NV <= 4 * NS, "the field table must fit in the staging area");
    __shared__ R smem[4 * NS];
    R(*stg)[NS] = reinterpret_cast<R(*)[NS]>(smem);  // D_x D_y D_z phi, then S_x S_y S_z
    R(*sF)[NV] = reinterpret_cast<R(*)[NV]>(smem);
    // Tiles away from the x ends of the mesh load each box row as aligned
    // 16-byte vectors over [L-VW, L+8+VW) (VW values per vector): fewer,
    // wider load instructions for a few more bytes.  Other tiles load point
    // by point with wrapped or clamped indices.
    constexpr int VW = 16 / (int)sizeof(R);
    constexpr int NVR = 8 / VW + 2;               // vectors per box row
    constexpr int NIT = SG * SG * NVR;            // vectors per array
    constexpr int NVE = (NIT + BLOCK - 1) / BLOCK;
    typedef R V __attribute__((ext_vector_type(VW)));
    const bool vec = S.n[0] % VW == 0 && S.cell0 % VW == 0 && L0 >= VW && L0 + 8 + VW <= S.n[0];
    R ssum[3][NSE];
    V vsum[3][NVE];
    int vrow[NVE], vvi[NVE];
    {
        const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
        const long long l0 = step % 3, l1 = (step + 1) % 3;
        if (vec) {
            V v0[3][NVE], v1[3][NVE], vp[NVE];
#pragma unroll
            for (int m = 0; m < NVE; ++m) {
                const int it = threadIdx.x + m * BLOCK;
                vrow[m] = it / NVR;
                vvi[m] = it % NVR;
                if (it < NIT) {
                    const int gj = axis_index(L1 - 1 + vrow[m] % SG, ny, S.bc[1]);
                    const int gkk = axis_index(L2 - 1 + vrow[m] / SG, nz, S.bc[2]);
                    const long long g =
                        ((long long)gkk * ny + gj) * nx + (L0 - VW + vvi[m] * VW) + S.cell0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        v0[c][m] = *reinterpret_cast<const V *>((const R *)ar.pot[l0][c] + g);
                        v1[c][m] = *reinterpret_cast<const V *>((const R *)ar.pot[l1][c] + g);
                    }
                    vp[m] = *reinterpret_cast<const V *>((const R *)ar.pot[l0][3] + g);
                }
            }
#pragma unroll
            for (int m = 0; m < NVE; ++m) {
                const int it = threadIdx.x + m * BLOCK;
                if (it < NIT) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) vsum[c][m] = v0[c][m] + v1[c][m];
#pragma unroll
                    for (int k = 0; k < VW; ++k) {
                        const int rx = vvi[m] * VW + k - VW + 1;  // box x index
                        if (rx >= 0 && rx < SG) {
                            const int e = vrow[m] * SG + rx;
#pragma unroll
                            for (int c = 0; c < 3; ++c) stg[c][e] = v1[c][m][k] - v0[c][m][k];
                            stg[3][e] = vp[m][k];
                        }
                    }
                }
            }
        } else {
            R a0[3][NSE], a1[3][NSE], ph[NSE];
#pragma unroll
            for (int m = 0; m < NSE; ++m) {
                const int e = threadIdx.x + m * BLOCK;
                if (e < NS) {
                    const int r0 = e % SG, r1 = (e / SG) % SG, r2 = e / (SG * SG);
                    const int gi = axis_index(L0 - 1 + r0, nx, S.bc[0]);
                    const int gj = axis_index(L1 - 1 + r1, ny, S.bc[1]);
                    const int gkk = axis_index(L2 - 1 + r2, nz, S.bc[2]);
                    const long long g = ((long long)gkk * ny + gj) * nx + gi;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        a0[c][m] = ((const R *)ar.pot[l0][c] + S.cell0)[g];
                        a1[c][m] = ((const R *)ar.pot[l1][c] + S.cell0)[g];
                    }
                    ph[m] = ((const R *)ar.pot[l0][3] + S.cell0)[g];
                }
            }
#pragma unroll
            for (int m = 0; m < NSE; ++m) {
                const int e = threadIdx.x + m * BLOCK;
#pragma unroll
                for (int c = 0; c < 3; ++c) ssum[c][m] = (R)0;
                if (e < NS) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        ssum[c][m] = a0[c][m] + a1[c][m];
                        stg[c][e] = a1[c][m] - a0[c][m];
                    }
                    stg[3][e] = ph[m];
                }
            }
        }
    }
    __syncthreads();
    {
        const R kE = (R)S.kE, kB = (R)S.kB;
        const R hidt = (R)(0.5 * S.inv_dt);
        const R q2x = (R)(0.25 * S.inv_2d[0]), q2y = (R)(0.25 * S.inv_2d[1]),
                q2z = (R)(0.25 * S.inv_2d[2]);
        const R i2x = (R)S.inv_2d[0], i2y = (R)S.inv_2d[1], i2z = (R)S.inv_2d[2];
        R EB[VPT][6];
        bool ok[VPT];
        int pp[VPT];
#pragma unroll
        for (int m = 0; m < VPT; ++m) {
            const int v = threadIdx.x + m * BLOCK;
            const int vi = v % TILE_VERT, vj = (v / TILE_VERT) % TILE_VERT,
                      vk = v / (TILE_VERT * TILE_VERT);
            ok[m] = v < NV && vertex_valid(S, L0 + vi, L1 + vj, L2 + vk);
            pp[m] = ((vk + 1) * SG + (vj + 1)) * SG + (vi + 1);
#pragma unroll
            for (int a = 0; a < 6; ++a) EB[m][a] = (R)0;
            if (ok[m]) {
                const int p = pp[m];
                const R *Dx = stg[0], *Dy = stg[1], *Dz = stg[2], *P = stg[3];
                // E = -dA/dt - grad phi
                EB[m][0] = -hidt * (Dx[p] + Dx[p - OX]) - (P[p + OX] - P[p - OX]) * i2x;
                EB[m][1] = -hidt * (Dy[p] + Dy[p - OY]) - (P[p + OY] - P[p - OY]) * i2y;
                EB[m][2] = -hidt * (Dz[p] + Dz[p - OZ]) - (P[p + OZ] - P[p - OZ]) * i2z;
            }
        }
        __syncthreads();  // the level sums overwrite the differences
        if (vec) {
#pragma unroll
            for (int m = 0; m < NVE; ++m) {
                const int it = threadIdx.x + m * BLOCK;
                if (it < NIT) {
#pragma unroll
                    for (int k = 0; k < VW; ++k) {
                        const int rx = vvi[m] * VW + k - VW + 1;
                        if (rx >= 0 && rx < SG) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) stg[c][vrow[m] * SG + rx] = vsum[c][m][k];
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int m = 0; m < NSE; ++m) {
                const int e = threadIdx.x + m * BLOCK;
                if (e < NS) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) stg[c][e] = ssum[c][m];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < VPT; ++m) {
            if (ok[m]) {
                const int p = pp[m];
                const R *Sx = stg[0], *Sy = stg[1], *Sz = stg[2];
                // B = mean over the two levels of curl A
                EB[m][3] = q2y * ((Sz[p + OY] + Sz[p + OY - OZ]) - (Sz[p - OY] + Sz[p - OY - OZ])) -
                           q2z * ((Sy[p + OZ] + Sy[p + OZ - OY]) - (Sy[p - OZ] + Sy[p - OZ - OY]));
                EB[m][4] = q2z * ((Sx[p + OZ] + Sx[p + OZ - OX]) - (Sx[p - OZ] + Sx[p - OZ - OX])) -
                           q2x * ((Sz[p + OX] + Sz[p + OX - OZ]) - (Sz[p - OX] + Sz[p - OX - OZ]));
                EB[m][5] = q2x * ((Sy[p + OX] + Sy[p + OX - OY]) - (Sy[p - OX] + Sy[p - OX - OY])) -
                           q2y * ((Sx[p + OY] + Sx[p + OY - OX]) - (Sx[p - OY] + Sx[p - OY - OX]));
            }
        }
        __syncthreads();  // the field table overwrites the staging buffers
#pragma unroll
        for (int m = 0; m < VPT; ++m) {
            const int v = threadIdx.x + m * BLOCK;
            if (v >= NV) continue;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                sF[a][v] = kE * EB[m][a];
                sF[3 + a][v] = kB * EB[m][3 + a];
            }
        }
    }
    __syncthreads();

    R *__restrict__ q0 = (R *)ar.ooff[0];
    R *__restrict__ q1 = (R *)ar.ooff[1];
    R *__restrict__ q2 = (R *)ar.ooff[2];
    const bool want_ke = S.mesh_every > 0 && ((step + 1) % S.mesh_every) == 0;
    const double t0 = ((double)step + 0.5) * S.dt;

    // uniform trip count over the block: count_runs needs whole wavefronts
    for (int base = p_lo; base < p_hi; base += BLOCK) {
        const int p = base + threadIdx.x;
        const bool active = p < p_hi;
        int ngk = 0;
        if (active) {
            if (!PRELOAD || base != p_lo) {
                gk = key[p];
                f[0] = o0[p];
                f[1] = o1[p];
                f[2] = o2[p];
                u[0] = u0[p];
                u[1] = u1[p];
                u[2] = u2[p];
            }
            const int lkey = (gk - (int)S.key0) & (TILE_CELLS - 1);
            const int li = lkey & 7, lj = (lkey >> 3) & 7, lk = lkey >> 6;
            int c[3] = {L0 + li, L1 + lj, L2 + lk};
            q0[p] = f[0];
            q1[p] = f[1];
            q2[p] = f[2];
            // linear interpolation of the 6 kick-scaled components from LDS
            R F[6];
            {
                const int b = (lk * TILE_VERT + lj) * TILE_VERT + li;
                const R wx1 = f[0], wx0 = (R)1 - f[0], wy1 = f[1], wy0 = (R)1 - f[1];
                const R wz1 = f[2], wz0 = (R)1 - f[2];
                constexpr int DY = TILE_VERT, DZ = TILE_VERT * TILE_VERT;
#pragma unroll
                for (int a = 0; a < 6; ++a) {
                    const R *g = sF[a];
                    const R x00 = wx0 * g[b] + wx1 * g[b + 1];
                    const R x10 = wx0 * g[b + DY] + wx1 * g[b + DY + 1];
                    const R x01 = wx0 * g[b + DZ] + wx1 * g[b + DZ + 1];
                    const R x11 = wx0 * g[b + DZ + DY] + wx1 * g[b + DZ + DY + 1];
                    F[a] = wz0 * (wy0 * x00 + wy1 * x10) + wz1 * (wy0 * x01 + wy1 * x11);
                }
            }
            const double ph_cell0 = S.kz_cell * (double)c[2] + S.phase_off;
            for (int sub = 0; sub < S.nsub; ++sub) {
                const double ts = t0 + sub * S.dtb;
                const double y = S.origin[1] + ((double)c[1] + (double)f[1]) * S.d[1];
                R Eu, Buy, Buz, Euy = 0, Bux = 0;
                if (OPTICAL && S.opt_on && S.opt_beam == 1) {
                    const double x = S.origin[0] + ((double)c[0] + (double)f[0]) * S.d[0];
                    const double z = S.origin[2] + ((double)c[2] + (double)f[2]) * S.d[2];
                    double E[2], B[3];
                    optical_gaussian_beam(S, ts, x, y, z, E, B);
                    Eu = (R)(S.kE * E[0]);
                    Euy = (R)(S.kE * E[1]);
                    Bux = (R)(S.kB * B[0]);
                    Buy = (R)(S.kB * B[1]);
                    Buz = (R)(S.kB * B[2]);
                } else if (OPTICAL && S.opt_on) {
                    // optical undulator: E = -a p s', B = (-a p_y s', a p_x s') / c
                    const double z = S.origin[2] + ((double)c[2] + (double)f[2]) * S.d[2];
                    const double ds = optical_rate(S, ts + (z - S.opt_zref) / C_LIGHT_D);
                    Eu = (R)(-S.kE * S.opt_p[0] * ds);
                    Euy = (R)(-S.kE * S.opt_p[1] * ds);
                    Bux = (R)(-S.kB * S.opt_p[1] * ds / C_LIGHT_D);
                    Buy = (R)(S.kB * S.opt_p[0] * ds / C_LIGHT_D);
                    Buz = 0;
                } else {
                    undulator_kick<R>(S, ph_cell0 + S.phase_rate * ts, f[2], y, Eu, Buy, Buz);
                }
                const R e0 = F[0] + Eu, e1 = F[1] + Euy, e2 = F[2];
                const R b0 = F[3] + Bux, b1 = F[4] + Buy, b2 = F[5] + Buz;
                // Boris: half kick, rotation, half kick
                const R t1x = u[0] + e0, t1y = u[1] + e1, t1z = u[2] + e2;
                const R ig = (R)1 / sqrt((R)1 + t1x * t1x + t1y * t1y + t1z * t1z);
                const R bx = b0 * ig, by = b1 * ig, bz = b2 * ig;
                const R t2x = t1x + (t1y * bz - t1z * by);
                const R t2y = t1y + (t1z * bx - t1x * bz);
                const R t2z = t1z + (t1x * by - t1y * bx);
                const R fac = (R)2 / ((R)1 + bx * bx + by * by + bz * bz);
                const R wx = fac * bx, wy = fac * by, wz = fac * bz;
                u[0] = t1x + (t2y * wz - t2z * wy) + e0;
                u[1] = t1y + (t2z * wx - t2x * wz) + e1;
                u[2] = t1z + (t2x * wy - t2y * wx) + e2;
                const R ginv = (R)1 / sqrt((R)1 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                f[0] += (R)S.cdtb_d[0] * u[0] * ginv;
                f[1] += (R)S.cdtb_d[1] * u[1] * ginv;
                f[2] += (R)S.cdtb_d[2] * u[2] * ginv;
            }
            bool ok = isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(f[0]) &&
                      isfinite(f[1]) && isfinite(f[2]);
            int nk = (int)S.nkeys;
            // record of the start cell for the deposit: x inside the tile and
            // the cell move per axis (-1, 0, 1; a move is below one cell)
            int move = li;
            if (ok) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const R fl = floor(f[a]);
                    c[a] += (int)fl;
                    f[a] -= fl;
                    move |= ((int)fl + 1) << (3 + 2 * a);
                    if (c[a] < 2 || c[a] > S.n[a] - 3) ok = false;  // lost
                }
                if (ok) nk = tile_key(S, c[0], c[1], c[2]);
            } else {
                atomicOr(&ar.flags[it.x], 1);
            }
            ar.okey[p] = ok ? move : OKEY_LOST;
            ngk = (int)S.key0 + nk;
            key[p] = ngk;
            o0[p] = f[0];
            o1[p] = f[1];
            o2[p] = f[2];
            u0[p] = u[0];
            u1[p] = u[1];
            u2[p] = u[2];
            if (!ok || want_ke) {
                const int pid = ar.id[par][p];
                double ke = 0.0;
                if (ok)
                    ke = sqrt(1.0 + (double)u[0] * u[0] + (double)u[1] * u[1] +
                              (double)u[2] * u[2]) -
                         1.0;
                ar.ke[S.part0 + pid] = ke;
                ar.zr[S.part0 + pid] =
                    ok ? S.origin[2] + ((double)c[2] + (double)f[2]) * S.d[2] : __builtin_nan("");
            }
        }
        count_runs(ar.counts, ngk, active);
        // flag the tiles this wavefront's particles entered (one write per
        // run of equal tiles)
        const int nloc = ngk - (int)S.key0;
        const bool inside = active && nloc < S.nkeys;
        const int ntile = inside ? S.tile0 + (nloc >> 9) : -1;
        const int prev = __shfl_up(ntile, 1);
        if (inside && ((threadIdx.x & 63) == 0 || prev != ntile)) ar.pocc[par ^ 1][ntile] = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && it.y != 0) ar.pocc[par][ti] = 0;  // set again by a later push
}

// ---------------------------------------------------------------------------
// 4. charge and current deposition (section "Current Deposition",
//    eq. (currentIntegral)) with Esirkepov's decomposition of the change of
//    the linear-weight density, which makes the discrete continuity equation
//    exact.  One block owns the 8^3 vertices of a tile and visits every
//    particle whose start cell lies in [L-2, L+8] per axis (those are all the
//    particles that can reach the tile), adding only what lands on its own
//    vertices.  A tile with no particle in its 27-tile neighbourhood has zero
//    sources; it writes them only when per-tile flags say they are not zero
//    already, so only the bunch's neighbourhood costs memory traffic.
//    Sums are fixed point in LDS: each term t (|t| <= 1) is scaled by 2^S,
//    rounded to an integer and added to a 64-bit accumulator.  Integer
//    addition is associative, so the result does not depend on the order of
//    the atomics.  S is chosen per tile from the number of particles the tile
//    visits, S = min(50, 62 - ceil(log2(visits + 1))): no accumulator can
//    overflow, and the resolution is 2^-S of one particle's weight (2^-50 for
//    tiles below 4096 visits, finer than the rounding of the FP64 terms).
//    The flush converts once and writes every vertex, zeros included.
// ---------------------------------------------------------------------------

constexpr double FX_SHIFT = 0x1.8p52;                      // 1.5 * 2^52
constexpr long long FX_SHIFT_BITS = 0x4338000000000000LL;  // its bit pattern
constexpr int FX_MAX_BITS = 50;                            // 2^S < 2^51

// v rounded to the nearest integer (ties to even) for |v| < 2^51: adding
// 1.5 * 2^52 leaves the integer in the low mantissa bits
__device__ __forceinline__ long long fx_round(double v)
{
    return __double_as_longlong(__dadd_rn(v, FX_SHIFT)) - FX_SHIFT_BITS;
}

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_deposit(const SimDev *__restrict__ sims,
                                                    const Brick *__restrict__ bricks, int nbricks,
                                                    int4 bs, Arena ar, int init)
{
    // The tile table lists the tiles of all simulations in order, so the
    // entry index is the global tile index.  A tile with no particle in its
    // 27-tile neighbourhood (flag set by the push) has zero sources; it writes
    // them only if they still hold values from an earlier step.  The flags,
    // the table entry and the step counter are read in one round trip.  (The
    // first deposit after loading particles has no push before it and takes
    // every tile.)
    int sim, tl, tg;  // tg: the global tile index
    if (!brick_tile(blockIdx.x, bricks, nbricks, bs, sim, tl, tg)) return;
    const int act = ar.tact[tg];
    const int jd = ar.jdirty[tg], rd0 = ar.rdirty[0][tg], rd1 = ar.rdirty[1][tg];
    const int2 it = make_int2(sim, tl);
    const long long step = *ar.d_step;
    const int par = (int)(step & 1);
    const int dst = init ? par : par ^ 1;
    const bool zj = jd != 0, zr = (dst ? rd1 : rd0) != 0;
    if (!init && !act && !zj && !zr) return;

    const SimDev &S = sims[it.x];
    const int *__restrict__ offs = ar.offs[par];
    const int t = it.y;
    const int tX = t % S.nt[0], tY = (t / S.nt[0]) % S.nt[1], tZ = t / (S.nt[0] * S.nt[1]);
    const int L[3] = {tX * TILE, tY * TILE, tZ * TILE};
    R *J0 = (R *)ar.J[0] + S.cell0, *J1 = (R *)ar.J[1] + S.cell0, *J2 = (R *)ar.J[2] + S.cell0;
    R *rho = (R *)ar.rho[dst] + S.cell0;
    const long long sy = S.n[0], sz = (long long)S.n[0] * S.n[1];

    if (!init && !act) {
        for (int e = threadIdx.x; e < TILE_CELLS; e += BLOCK) {
            const int vx = L[0] + (e & 7), vy = L[1] + ((e >> 3) & 7), vz = L[2] + (e >> 6);
            if (vx >= S.n[0] || vy >= S.n[1] || vz >= S.n[2]) continue;
            const long long g = vz * sz + vy * sy + vx;
            if (zj) J0[g] = J1[g] = J2[g] = (R)0;
            if (zr) rho[g] = (R)0;
        }
        if (threadIdx.x == 0) {
            ar.jdirty[tg] = 0;
            ar.rdirty[dst][tg] = 0;
        }
        return;
    }

    constexpr int NENT = 363;  // 11 x 11 rows of start cells, up to 3 key ranges each
    constexpr int QCAP = 3 * BLOCK;
    __shared__ unsigned long long acc[4][TILE_CELLS];
    __shared__ int rstart[384], rpre[384];
    // queues (0: particles that stay in their cell, 1: the others): particle
    // index, packed start cell and move
    __shared__ int qp[2][QCAP], qi[2][QCAP];
    __shared__ int wsum[BLOCK / 64];
    __shared__ int qn[2];

    // particle ranges: rows of start cells (y, z) in [L-2, L+8], x-range
    // [L-2, L+8] split at tile boundaries (at most 3 contiguous key ranges)
    int mylen[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = threadIdx.x * 2 + h;
        int st = 0, ln = 0;
        if (e < NENT) {
            const int row = e / 3, piece = e % 3;
            const int cy = L[1] - 2 + row % 11, cz = L[2] - 2 + row / 11;
            const int xa = max(L[0] - 2, 0), xb = min(L[0] + 8, S.n[0] - 1);
            const int tx = tX - 1 + piece;
            const int pa = max(xa, tx * TILE), pb = min(xb, tx * TILE + TILE - 1);
            if (cy >= 0 && cy < S.n[1] && cz >= 0 && cz < S.n[2] && tx >= 0 && tx < S.nt[0] &&
                pa <= pb) {
                const long long ka = S.key0 + tile_key(S, pa, cy, cz);
                const long long kb = S.key0 + tile_key(S, pb, cy, cz);
                st = offs[ka];
                ln = offs[kb + 1] - st;
            }
            rstart[e] = st;
        }
        mylen[h] = ln;
    }
    for (int e = threadIdx.x; e < 4 * TILE_CELLS; e += BLOCK) (&acc[0][0])[e] = 0ull;
    if (threadIdx.x < 2) qn[threadIdx.x] = 0;
    int total;
    const int pre = block_excl_scan(mylen[0] + mylen[1], wsum, &total);
    if (threadIdx.x * 2 < NENT) rpre[threadIdx.x * 2] = pre;
    if (threadIdx.x * 2 + 1 < NENT) rpre[threadIdx.x * 2 + 1] = pre + mylen[0];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    // fixed-point scale of this tile: at most `total` terms meet at a vertex
    const int fx_bits = min(FX_MAX_BITS, 62 - (32 - __clz(total)));
    const double scale = ldexp(1.0, fx_bits);
    const R *__restrict__ n0 = (const R *)ar.off[par][0];
    const R *__restrict__ n1 = (const R *)ar.off[par][1];
    const R *__restrict__ n2 = (const R *)ar.off[par][2];
    const R *__restrict__ q0 = init ? n0 : (const R *)ar.ooff[0];
    const R *__restrict__ q1 = init ? n1 : (const R *)ar.ooff[1];
    const R *__restrict__ q2 = init ? n2 : (const R *)ar.ooff[2];

    // terms off the tile and zero terms are skipped
    auto add = [&](int q, bool own, int e, double t) __attribute__((always_inline)) {
        if (!own) return;
        const long long v = fx_round(__dmul_rn(t, scale));  // scaling is exact
        if (v) atomicAdd(&acc[q][e], (unsigned long long)v);
    };

    // One queued particle: its start cell and move (packed by the filter) and
    // its start and end positions inside the cells.  For a particle that
    // stays in its cell (nm true) the weights on the far vertex of each axis
    // are zero and the loops over them are left out; the terms kept are the
    // same expressions as in the general case.
    auto deposit_one = [&](auto nm, int p, int info) __attribute__((always_inline)) {
        constexpr bool NM = decltype(nm)::value;
        constexpr int NB = NM ? 2 : 3;
        const R f0[3] = {q0[p], q1[p], q2[p]};
        const R f1[3] = {n0[p], n1[p], n2[p]};
        int base[3];
        bool moved[3];
        R S0[3][3], DS[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int c0 = ((info >> (4 * a)) & 15) - 2;        // start cell - L
            const int mv = NM ? 0 : ((info >> (12 + 2 * a)) & 3) - 1;  // cell move
            moved[a] = mv != 0;
            base[a] = min(c0, c0 + mv);
            // the start (end) cell is base or base + 1
            const bool s0 = mv >= 0, s1 = mv <= 0;
            R S1[3];
            S0[a][0] = s0 ? (R)1 - f0[a] : (R)0;
            S0[a][1] = s0 ? f0[a] : (R)1 - f0[a];
            S0[a][2] = s0 ? (R)0 : f0[a];
            S1[0] = s1 ? (R)1 - f1[a] : (R)0;
            S1[1] = s1 ? f1[a] : (R)1 - f1[a];
            S1[2] = s1 ? (R)0 : f1[a];
#pragma unroll
            for (int m = 0; m < 3; ++m) DS[a][m] = S1[m] - S0[a][m];
        }
        // the 3x3x3 box [base, base+2] in tile-local vertex coordinates;
        // J_l sits on the edges from vertex a to a + 1 along l (a = 0, 1).
        // Without a move along l the weights along l sit on two vertices and
        // the current on the second edge is DS_0 + DS_1 = -DS_2 = 0 exactly;
        // only its rounding residue would remain, so it is not added.
        auto own = [](int v) { return v >= 0 && v < TILE; };
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const int pa = (l + 1) % 3, ra = (l + 2) % 3;
#pragma unroll
            for (int bb = 0; bb < NB; ++bb)
#pragma unroll
                for (int ee = 0; ee < NB; ++ee) {
                    const R Y = S0[pa][bb] * S0[ra][ee] + (R)0.5 * DS[pa][bb] * S0[ra][ee] +
                                (R)0.5 * S0[pa][bb] * DS[ra][ee] +
                                DS[pa][bb] * DS[ra][ee] * (R)(1.0 / 3.0);
                    R run = 0;
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        if (a == 1 && (NM || !moved[l])) break;
                        run += DS[l][a] * Y;
                        int v[3];
                        v[l] = base[l] + a;
                        v[pa] = base[pa] + bb;
                        v[ra] = base[ra] + ee;
                        add(l, own(v[0]) && own(v[1]) && own(v[2]),
                            (v[2] * TILE + v[1]) * TILE + v[0], (double)run);
                    }
                }
        }
        // rho^{s+3/2} at the 8 vertices of the end cell
        int e1[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            e1[a] = ((info >> (4 * a)) & 15) - 2 + (NM ? 0 : ((info >> (12 + 2 * a)) & 3) - 1);
#pragma unroll
        for (int K = 0; K < 2; ++K)
#pragma unroll
            for (int J = 0; J < 2; ++J)
#pragma unroll
                for (int I = 0; I < 2; ++I) {
                    const int vx = e1[0] + I, vy = e1[1] + J, vz = e1[2] + K;
                    const R w8 = (I ? f1[0] : (R)1 - f1[0]) * (J ? f1[1] : (R)1 - f1[1]) *
                                 (K ? f1[2] : (R)1 - f1[2]);
                    add(3, own(vx) && own(vy) && own(vz), (vz * TILE + vy) * TILE + vx,
                        (double)w8);
                }
    };

    // Candidates in chunks of one per thread.  The filter reads only the
    // 4-byte move record, keeps the particles whose vertex support
    // [min(c0, c1), max(c0, c1) + 1] meets the tile on every axis, and
    // appends them to an LDS queue; a full block's worth is deposited at a
    // time.  The queue order varies between runs, the integer sums do not.
    const int *__restrict__ okey = ar.okey;
    const int *__restrict__ key = ar.key[par];
    // the candidate's range, particle index and move record
    auto locate = [&](int w, int *lo_out) __attribute__((always_inline)) {
        int lo = 0, hi = NENT - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rpre[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        *lo_out = lo;
        return rstart[lo] + (w - rpre[lo]);
    };
    auto record = [&](int p) __attribute__((always_inline)) {
        if (!init) return okey[p];
        const int nk = key[p] - (int)S.key0;
        return nk >= S.nkeys ? OKEY_LOST : (nk & 7) | (0x15 << 3);  // no move
    };
    // keep the particle if its vertex support meets the tile; packs the
    // start cell relative to the tile (+2, 4 bits per axis) and the move
    // (+1, 2 bits per axis)
    auto filter = [&](int lo, int rec, int *info) __attribute__((always_inline)) {
        *info = 0;
        if (rec & OKEY_LOST) return false;
        const int row = lo / 3;
        const int c0[3] = {(tX - 1 + lo % 3) * TILE + (rec & 7) - L[0], row % 11 - 2,
                           row / 11 - 2};
        bool take = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int mv = ((rec >> (3 + 2 * a)) & 3) - 1;
            const int mn = min(c0[a], c0[a] + mv), mx = max(c0[a], c0[a] + mv);
            take = take && mx + 1 >= 0 && mn <= TILE - 1;
            *info |= (c0[a] + 2) << (4 * a) | (mv + 1) << (12 + 2 * a);
        }
        return take;
    };
    auto append = [&](bool take, int p, int info) __attribute__((always_inline)) {
        const bool still = (info >> 12) == 0x15;  // no move on any axis
#pragma unroll
        for (int Q = 0; Q < 2; ++Q) {
            const bool mine = take && (still == (Q == 0));
            const unsigned long long m = __ballot(mine);
            int wbase = 0;
            if (lane == 0 && m) wbase = atomicAdd(&qn[Q], __popcll(m));
            wbase = __shfl(wbase, 0);
            if (mine) {
                const int pos = wbase + __popcll(m & ((1ull << lane) - 1ull));
                qp[Q][pos] = p;
                qi[Q][pos] = info;
            }
        }
    };
    // Candidates in chunks of two per thread.  The filter reads only the
    // 4-byte move record; the kept particles wait in LDS queues and are
    // deposited a full block at a time (taken from the end of the queue).
    // The order varies between runs, the integer sums do not.
    for (int g = 0; g < total; g += 2 * BLOCK) {
        const int wa = g + threadIdx.x, wb = wa + BLOCK;
        int la = 0, lb = 0, pa = 0, pb = 0, ra = OKEY_LOST, rb = OKEY_LOST;
        if (wa < total) pa = locate(wa, &la);
        if (wb < total) pb = locate(wb, &lb);
        if (wa < total) ra = record(pa);
        if (wb < total) rb = record(pb);
        int ia, ib;
        const bool ta = filter(la, ra, &ia), tb = filter(lb, rb, &ib);
        append(ta, pa, ia);
        append(tb, pb, ib);
        __syncthreads();
        const bool last = g + 2 * BLOCK >= total;
        auto drain = [&](auto nm) __attribute__((always_inline)) {
            constexpr int Q = decltype(nm)::value ? 0 : 1;
            for (;;) {
                const int n = qn[Q];
                if (last ? n == 0 : n < BLOCK) break;  // uniform
                const int cnt = min(n, BLOCK);
                const bool has = (int)threadIdx.x < cnt;
                int p = 0, info = 0;
                if (has) {
                    p = qp[Q][n - cnt + threadIdx.x];
                    info = qi[Q][n - cnt + threadIdx.x];
                }
                __syncthreads();
                if (threadIdx.x == 0) qn[Q] = n - cnt;
                if (has) deposit_one(nm, p, info);
                __syncthreads();
            }
        };
        drain(std::integral_constant<bool, true>());
        drain(std::integral_constant<bool, false>());
        __syncthreads();
    }

    // flush: every owned vertex, zeros included
    if (threadIdx.x == 0) ar.tact[tg] = 0;  // set again by the next push
    const double inv = ldexp(1.0, -fx_bits);
    const double ju0 = S.J_unit[0] * inv, ju1 = S.J_unit[1] * inv, ju2 = S.J_unit[2] * inv,
                 ru = S.rho_unit * inv;
    if (threadIdx.x == 0) {
        ar.jdirty[tg] = 1;
        ar.rdirty[dst][tg] = 1;
    }
    for (int e = threadIdx.x; e < TILE_CELLS; e += BLOCK) {
        const int vx = L[0] + (e & 7), vy = L[1] + ((e >> 3) & 7), vz = L[2] + (e >> 6);
        if (vx >= S.n[0] || vy >= S.n[1] || vz >= S.n[2]) continue;
        const long long g = vz * sz + vy * sy + vx;
        J0[g] = (R)((double)(long long)acc[0][e] * ju0);
        J1[g] = (R)((double)(long long)acc[1][e] * ju1);
        J2[g] = (R)((double)(long long)acc[2][e] * ju2);
        rho[g] = (R)((double)(long long)acc[3][e] * ru);
    }
}

// ---------------------------------------------------------------------------
// 5. exclusive scan of the bucket counts -> bucket starts (offs[(s+1) & 1]).
//    Reduce per chunk, scan the chunk sums in one block, then scan each chunk
//    with its base.  Wavefront scans use cross-lane shuffles.
// ---------------------------------------------------------------------------

// A chunk is SCAN_CHUNK / SCAN_ROW rows of SCAN_ROW keys; in a row, thread t
// holds keys 4t .. 4t+3, so every load and store instruction is one
// contiguous 1 KB span per wavefront.
constexpr int SCAN_ROW = BLOCK * 4;
static_assert(SCAN_CHUNK % SCAN_ROW == 0, "a chunk is whole rows");

__device__ __forceinline__ int4 load4(const int *__restrict__ a, long long i, long long n)
{
    if (i + 3 < n) return *reinterpret_cast<const int4 *>(a + i);
    int4 v = make_int4(0, 0, 0, 0);
    if (i < n) v.x = a[i];
    if (i + 1 < n) v.y = a[i + 1];
    if (i + 2 < n) v.z = a[i + 2];
    return v;
}

// A chunk of keys whose tiles no particle can occupy in the next step (their
// occupancy flags, written by the push, are clear) and that holds no lost
// bucket has only zero counts: the scan skips reading them.  chunks[b] =
// (first global tile, last global tile, holds a lost bucket); the flags of
// the next step are pocc[(step + 1) & 1].  Uniform over the block.
__device__ __forceinline__ bool chunk_empty(const int4 *__restrict__ chunks, const Arena &ar)
{
    __shared__ int any;
    const int4 ck = chunks[blockIdx.x];
    const long long step = *ar.d_step;
    const int *__restrict__ occ = ar.pocc[(step + 1) & 1];
    if (threadIdx.x == 0) any = ck.z;
    __syncthreads();
    const int t = ck.x + (int)threadIdx.x;
    if (t <= ck.y && occ[t]) any = 1;
    __syncthreads();
    const bool empty = any == 0;
    __syncthreads();  // every thread has read the flag
    return empty;
}

__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const int *__restrict__ counts,
                                                        long long n, int *__restrict__ bsum,
                                                        const int4 *__restrict__ chunks, Arena ar)
{
    if (chunk_empty(chunks, ar)) {
        if (threadIdx.x == 0) bsum[blockIdx.x] = 0;
        return;
    }
    const long long base = (long long)blockIdx.x * SCAN_CHUNK + 4 * threadIdx.x;
    int4 v[SCAN_CHUNK / SCAN_ROW];
#pragma unroll
    for (int r = 0; r < SCAN_CHUNK / SCAN_ROW; ++r) v[r] = load4(counts, base + r * SCAN_ROW, n);
    int s = 0;
#pragma unroll
    for (int r = 0; r < SCAN_CHUNK / SCAN_ROW; ++r) s += v[r].x + v[r].y + v[r].z + v[r].w;
    __shared__ int sh[BLOCK / 64];
    int tot;
    block_excl_scan(s, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// One block: exclusive scan of the chunk sums, TOP_SEG at a time, staged
// through LDS (padded by one word per 32 so that each thread's consecutive
// run lies in distinct banks).
constexpr int TOP_PER_THREAD = 32;
constexpr int TOP_SEG = BLOCK * TOP_PER_THREAD;

__global__ __launch_bounds__(BLOCK) void k_scan_top(int *__restrict__ bsum, int nb)
{
    __shared__ int seg[TOP_SEG + TOP_SEG / 32];
    __shared__ int sh[BLOCK / 64];
    auto pad = [](int j) { return j + (j >> 5); };
    int carry = 0;
    for (int base = 0; base < nb; base += TOP_SEG) {
        for (int j = threadIdx.x; j < TOP_SEG; j += BLOCK)
            seg[pad(j)] = base + j < nb ? bsum[base + j] : 0;
        __syncthreads();
        const int j0 = threadIdx.x * TOP_PER_THREAD;
        int s = 0;
#pragma unroll
        for (int k = 0; k < TOP_PER_THREAD; ++k) s += seg[pad(j0 + k)];
        int tot;
        int run = carry + block_excl_scan(s, sh, &tot);
#pragma unroll
        for (int k = 0; k < TOP_PER_THREAD; ++k) {
            const int v = seg[pad(j0 + k)];
            seg[pad(j0 + k)] = run;
            run += v;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < TOP_SEG && base + j < nb; j += BLOCK)
            bsum[base + j] = seg[pad(j)];
        carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(BLOCK) void k_scan_down(const int *__restrict__ counts, long long n,
                                                      const int *__restrict__ bsum,
                                                      const int4 *__restrict__ chunks, Arena ar)
{
    const long long step = *ar.d_step;
    int *__restrict__ out = ar.offs[(step + 1) & 1];
    const long long chunk0 = (long long)blockIdx.x * SCAN_CHUNK;
    const long long base = chunk0 + 4 * threadIdx.x;
    if (chunk_empty(chunks, ar)) {
        // every count is zero: each start is the carry into the chunk
        const int carry = bsum[blockIdx.x];
        const int4 o = make_int4(carry, carry, carry, carry);
#pragma unroll
        for (int r = 0; r < SCAN_CHUNK / SCAN_ROW; ++r) {
            const long long i = base + r * SCAN_ROW;
            if (i + 3 < n) {
                *reinterpret_cast<int4 *>(out + i) = o;
            } else {
                if (i < n) out[i] = carry;
                if (i + 1 < n) out[i + 1] = carry;
                if (i + 2 < n) out[i + 2] = carry;
            }
        }
        if (threadIdx.x == 0 && chunk0 + SCAN_CHUNK >= n) out[n] = carry;  // total
        return;
    }
    int4 v[SCAN_CHUNK / SCAN_ROW];
#pragma unroll
    for (int r = 0; r < SCAN_CHUNK / SCAN_ROW; ++r) v[r] = load4(counts, base + r * SCAN_ROW, n);
    __shared__ int sh[BLOCK / 64];
    int carry = bsum[blockIdx.x];
#pragma unroll
    for (int r = 0; r < SCAN_CHUNK / SCAN_ROW; ++r) {
        int tot;
        const int ex = block_excl_scan(v[r].x + v[r].y + v[r].z + v[r].w, sh, &tot);
        int4 o;
        o.x = carry + ex;
        o.y = o.x + v[r].x;
        o.z = o.y + v[r].y;
        o.w = o.z + v[r].z;
        const long long i = base + r * SCAN_ROW;
        if (i + 3 < n) {
            *reinterpret_cast<int4 *>(out + i) = o;
        } else {
            if (i < n) out[i] = o.x;
            if (i + 1 < n) out[i + 1] = o.y;
            if (i + 2 < n) out[i + 2] = o.z;
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && chunk0 + SCAN_CHUNK >= n) out[n] = carry;  // total
}

// ---------------------------------------------------------------------------
// 6. scatter to the new sorted order (buffer (s+1) & 1).  The slot inside a
//    bucket comes from an atomic decrement, which also returns the counts to
//    zero for the next step.  The order inside a cell is arbitrary; nothing
//    downstream depends on it (deposits are integer sums, the kinetic energy
//    is summed by particle id).
// ---------------------------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_scatter(Arena ar, long long np)
{
    // each XCD takes one contiguous range of particles, so the lines where
    // the destination ranges of neighbouring blocks meet are completed in one L2
    const long long p = (long long)xcd_remap(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    const bool active = p < np;  // every lane stays: the run logic is per wavefront
    const long long step = *ar.d_step;
    const int s = (int)(step & 1), d = s ^ 1;
    const int lane = threadIdx.x & 63;
    // All loads are issued up front, unconditionally (lanes past the end read
    // the last particle), so none waits for another: the payload before any
    // store, since the compiler cannot know that the source and destination
    // buffers are distinct, and the bucket start while the atomic is in flight.
    const long long pp = active ? p : np - 1;
    const int gk = ar.key[s][pp];
    const int pid = ar.id[s][pp];
    R po[3], pu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        po[a] = ((const R *)ar.off[s][a])[pp];
        pu[a] = ((const R *)ar.u[s][a])[pp];
    }
    const int start = ar.offs[d][gk];
    const int g = active ? gk : -1;
    const int prev = __shfl_up(g, 1, 64);
    const bool head = active && (lane == 0 || prev != g);
    const unsigned long long heads = __ballot(head);
    const unsigned long long act = __ballot(active);
    // one atomic per run of equal keys; the run takes the slots just below
    // the old count, in lane order
    int base = 0;
    if (head) {
        const unsigned long long later = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
        const int next = later ? __ffsll((long long)later) - 1 : 64;
        const unsigned long long span =
            (next == 64 ? ~0ull : ((1ull << next) - 1)) & (~0ull << lane);
        const int len = __popcll(act & span);
        base = atomicSub(&ar.counts[g], len) - len;
    }
    const unsigned long long upto = heads & ((2ull << lane) - 1);
    const int hl = upto ? 63 - __clzll((long long)upto) : 0;
    base = __shfl(base, hl, 64);
    if (!active) return;
    const int dst = start + base + __popcll(act & ((2ull << lane) - 1) & ~((1ull << hl) - 1)) - 1;
    ar.key[d][dst] = g;
    ar.id[d][dst] = pid;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ((R *)ar.off[d][a])[dst] = po[a];
        ((R *)ar.u[d][a])[dst] = pu[a];
    }
}

// ---------------------------------------------------------------------------
// 7. double-precision diagnostics.  Per-block partial sums in fixed order
//    (one launch: power-plane blocks, then mesh blocks, then kinetic-energy
//    blocks), then one block per simulation sums its partials in fixed order
//    and writes the row: deterministic run to run.  The last of those blocks
//    to finish advances the step counter.
// ---------------------------------------------------------------------------

// f = (E_x, E_y, B_x, B_y) of the bunch frame seen in the lab, where the frame
// moves along +z at beta0 c (section "Lorentz Transformation"); with
// G = gamma0 and GB = gamma0 beta0: E_x = G E_x + GB c B_y,
// E_y = G E_y - GB c B_x, B_x = G B_x - GB E_y / c, B_y = G B_y + GB E_x / c.
__device__ __forceinline__ void to_lab(const SimDev &S, const double f[4], double l[4])
{
    l[0] = S.lab_g * f[0] + S.lab_gb * C_LIGHT_D * f[3];
    l[1] = S.lab_g * f[1] - S.lab_gb * C_LIGHT_D * f[2];
    l[2] = S.lab_g * f[2] - S.lab_gb * f[1] / C_LIGHT_D;
    l[3] = S.lab_g * f[3] + S.lab_gb * f[0] / C_LIGHT_D;
}

template <typename R>
__device__ __forceinline__ void diag_plane(const SimDev *__restrict__ sims, int2 it, Arena &ar)
{
    // Per block of plane points: the Poynting flux in the bunch frame and in
    // the lab, and the running DFT of Ex, Ey, Bx, By at nu_f omega_1 advanced
    // by this step's sample at t = (s + 1/2) dt, with each point's
    // Re(F_Ex F_By* - F_Ey F_Bx*) in both frames.
    // item y = plate * nb_plane + block; plate 0 is the main plane (power, lab
    // power and spectrum), plates 1.. the further ones (power only)
    const SimDev &S = sims[it.x];
    const long long step = *ar.d_step;
    const FieldPtrs<R> f = field_ptrs<R>(S, ar, step % 3, (step + 1) % 3, (int)(step % 3));
    const int plate = it.y / S.nb_plane, blk = it.y - plate * S.nb_plane;
    const int kz = plate == 0 ? S.kp : S.kp_extra[plate - 1];
    const int e = blk * BLOCK + threadIdx.x;
    const long long npl = (long long)S.n[0] * S.n[1];
    double p0 = 0.0, pl = 0.0, fv[4] = {0.0, 0.0, 0.0, 0.0};
    bool valid = false;
    if (e < npl) {
        const int i = e % S.n[0], j = e / S.n[0];
        if (vertex_valid(S, i, j, kz)) {
            R E[3], B[3];
            vertex_EB<R>(S, f, i, j, kz, E, B);
            fv[0] = (double)E[0];
            fv[1] = (double)E[1];
            fv[2] = (double)B[0];
            fv[3] = (double)B[1];
            p0 = fv[0] * fv[3] - fv[1] * fv[2];
            double l[4];
            to_lab(S, fv, l);
            pl = l[0] * l[3] - l[1] * l[2];
            valid = true;
        }
    }
    __shared__ double sh[BLOCK];
    if (plate > 0) {
        const double tot = block_sum(p0, sh);
        if (threadIdx.x == 0)
            ar.partial[S.part_extra0 + (long long)(plate - 1) * S.nb_plane + blk] = tot;
        return;
    }
    double *o = ar.partial + S.part_plane0 + (long long)PLANE_STRIDE * blk;
    {
        const double t0 = block_sum(p0, sh);
        const double t1 = block_sum(pl, sh);
        if (threadIdx.x == 0) {
            o[0] = t0;
            o[1] = t1;
        }
    }
    if (!S.spec_on) return;  // uniform over the block
    // the sums are stored sum-major (sum q of point e at q * npl + e), so each
    // access is one contiguous span per wavefront; one frequency (8 sums) at
    // a time keeps the register count of the launch, which all roles share, low
    const double tm = ((double)step + 0.5) * S.dt;
    for (int fq = 0; fq < S.nfreq; ++fq) {  // uniform over the block
        double tr = 0.0, tl = 0.0;
        if (valid) {
            double sn, cs;
            sincos(S.fnu[fq] * S.omega1 * tm, &sn, &cs);
            double *af = ar.spec + S.spec0 + e + (long long)fq * SPEC_PER_FREQ * npl;
            double a[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) a[q] = af[q * npl];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                a[2 * c] = a[2 * c] + fv[c] * cs * S.dt;
                a[2 * c + 1] = a[2 * c + 1] - fv[c] * sn * S.dt;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) af[q * npl] = a[q];
            // (re, im) pairs: Ex a[0..1], Ey a[2..3], Bx a[4..5], By a[6..7]
            tr = (a[0] * a[6] + a[1] * a[7]) - (a[2] * a[4] + a[3] * a[5]);
            const double re[4] = {a[0], a[2], a[4], a[6]}, im[4] = {a[1], a[3], a[5], a[7]};
            double lr[4], li[4];
            to_lab(S, re, lr);
            to_lab(S, im, li);
            tl = (lr[0] * lr[3] + li[0] * li[3]) - (lr[1] * lr[2] + li[1] * li[2]);
        }
        const double sr = block_sum(tr, sh);
        const double sl = block_sum(tl, sh);
        if (threadIdx.x == 0) {
            o[2 + 2 * fq] = sr;
            o[3 + 2 * fq] = sl;
        }
    }
}

template <typename R>
__device__ __forceinline__ void diag_mesh(const SimDev *__restrict__ sims, int2 it, Arena &ar)
{
    const SimDev &S = sims[it.x];
    const long long step = *ar.d_step;
    if (S.mesh_every <= 0 || ((step + 1) % S.mesh_every) != 0) return;
    const FieldPtrs<R> f = field_ptrs<R>(S, ar, step % 3, (step + 1) % 3, (int)(step % 3));
    const R *rn = (const R *)ar.rho[(step + 1) & 1] + S.cell0;
    const R *ro = (const R *)ar.rho[step & 1] + S.cell0;
    const R *J0 = (const R *)ar.J[0] + S.cell0, *J1 = (const R *)ar.J[1] + S.cell0,
            *J2 = (const R *)ar.J[2] + S.cell0;
    const long long ncell = (long long)S.n[0] * S.n[1] * S.n[2];
    const long long sy = S.n[0], sz = (long long)S.n[0] * S.n[1];
    double q = 0.0, wf = 0.0, rmax = 0.0, res = 0.0;
    const long long base = (long long)it.y * BLOCK * MESH_DIAG_PER_THREAD;
    for (int r = 0; r < MESH_DIAG_PER_THREAD; ++r) {
        const long long g = base + (long long)r * BLOCK + threadIdx.x;
        if (g >= ncell) break;
        const int i = (int)(g % S.n[0]), j = (int)((g / S.n[0]) % S.n[1]), k = (int)(g / sz);
        const double rv = (double)rn[g];
        q += rv;
        rmax = fmax(rmax, fabs(rv));
        if (i >= 1 && j >= 1 && k >= 1) {
            const double div = ((double)J0[g] - (double)J0[g - 1]) / S.d[0] +
                               ((double)J1[g] - (double)J1[g - sy]) / S.d[1] +
                               ((double)J2[g] - (double)J2[g - sz]) / S.d[2];
            res = fmax(res, fabs(rv - (double)ro[g] + S.dt * div));
        }
        if (vertex_valid(S, i, j, k)) {
            R E[3], B[3];
            vertex_EB<R>(S, f, i, j, k, E, B);
            const double e2 = (double)E[0] * E[0] + (double)E[1] * E[1] + (double)E[2] * E[2];
            const double b2 = (double)B[0] * B[0] + (double)B[1] * B[1] + (double)B[2] * B[2];
            wf += S.eps0_half * e2 + S.inv_2mu0 * b2;
        }
    }
    __shared__ double sh[BLOCK];
    const double tq = block_sum(q, sh);
    const double tw = block_sum(wf, sh);
    const double tr = block_max(rmax, sh);
    const double ts = block_max(res, sh);
    if (threadIdx.x == 0) {
        double *o = ar.partial + S.part_mesh0 + 4 * (long long)it.y;
        o[0] = tq;
        o[1] = tw;
        o[2] = tr;
        o[3] = ts;
    }
}

// Per block of particle ids: sum (gamma - 1), the live count and the cos and
// sin sums of h K z for h = 1, 2, 3 (section "Bunching factor").  By id, so
// the order is fixed whatever the particles' order in memory; lost particles
// hold z = NaN.
__device__ __forceinline__ void diag_kin(const SimDev *__restrict__ sims, int2 it, Arena &ar)
{
    const SimDev &S = sims[it.x];
    const long long step = *ar.d_step;
    if (S.mesh_every <= 0 || ((step + 1) % S.mesh_every) != 0) return;
    double t[KIN_TERMS];
#pragma unroll
    for (int q = 0; q < KIN_TERMS; ++q) t[q] = 0.0;
    const long long base = (long long)it.y * BLOCK * KIN_PER_THREAD;
    for (int r = 0; r < KIN_PER_THREAD; ++r) {
        const long long i = base + (long long)r * BLOCK + threadIdx.x;
        if (i >= S.np) continue;
        t[0] += ar.ke[S.part0 + i];
        const double z = ar.zr[S.part0 + i];
        if (z == z) {
            t[1] += 1.0;
            // harmonics 2 and 3 of the phase by angle addition from the first
            double s1, c1;
            sincos(S.kbunch * z, &s1, &c1);
            const double c2 = c1 * c1 - s1 * s1, s2 = 2.0 * s1 * c1;
            t[2] += c1;
            t[3] += s1;
            t[4] += c2;
            t[5] += s2;
            t[6] += c2 * c1 - s2 * s1;
            t[7] += s2 * c1 + c2 * s1;
        }
    }
    __shared__ double sh[BLOCK];
#pragma unroll
    for (int q = 0; q < KIN_TERMS; ++q) {
        const double tot = block_sum(t[q], sh);
        if (threadIdx.x == 0) ar.partial[S.part_kin0 + (long long)KIN_TERMS * it.y + q] = tot;
    }
}

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_diag_parts(const SimDev *__restrict__ sims,
                                                       const int2 *__restrict__ plane, int nplane,
                                                       const int2 *__restrict__ mesh, int nmesh,
                                                       const int2 *__restrict__ kin, Arena ar)
{
    const int b = blockIdx.x;  // the role is uniform over the block
    if (b < nplane) diag_plane<R>(sims, plane[b], ar);
    else if (b < nplane + nmesh) diag_mesh<R>(sims, mesh[b - nplane], ar);
    else diag_kin(sims, kin[b - nplane - nmesh], ar);
}

template <typename R>
__global__ __launch_bounds__(BLOCK) void k_diag_final(const SimDev *__restrict__ sims, Arena ar)
{
    const SimDev &S = sims[blockIdx.x];
    const long long step = *ar.d_step;
    const bool mesh = S.mesh_every > 0 && ((step + 1) % S.mesh_every) == 0;
    __shared__ double sh[BLOCK];
    double pt[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < S.nb_plane; b += BLOCK) {
        const double *o = ar.partial + S.part_plane0 + (long long)PLANE_STRIDE * b;
        pt[0] += o[0];
        pt[1] += o[1];
    }
    pt[0] = block_sum(pt[0], sh);
    pt[1] = block_sum(pt[1], sh);
    const double pw = pt[0];
    double px[3] = {0.0, 0.0, 0.0};
    for (int p = 0; p < S.n_extra; ++p) {  // uniform over the block
        double v = 0.0;
        for (int b = threadIdx.x; b < S.nb_plane; b += BLOCK)
            v += ar.partial[S.part_extra0 + (long long)p * S.nb_plane + b];
        px[p] = block_sum(v, sh);
    }
    double q = 0.0, wf = 0.0, rmax = 0.0, res = 0.0, kt[KIN_TERMS];
#pragma unroll
    for (int t = 0; t < KIN_TERMS; ++t) kt[t] = 0.0;
    if (mesh) {
        for (int b = threadIdx.x; b < S.nb_mesh; b += BLOCK) {
            const double *o = ar.partial + S.part_mesh0 + 4 * (long long)b;
            q += o[0];
            wf += o[1];
            rmax = fmax(rmax, o[2]);
            res = fmax(res, o[3]);
        }
        for (int b = threadIdx.x; b < S.nb_kin; b += BLOCK) {
            const double *o = ar.partial + S.part_kin0 + (long long)KIN_TERMS * b;
#pragma unroll
            for (int t = 0; t < KIN_TERMS; ++t) kt[t] += o[t];
        }
        q = block_sum(q, sh);
        wf = block_sum(wf, sh);
        rmax = block_max(rmax, sh);
        res = block_max(res, sh);
#pragma unroll
        for (int t = 0; t < KIN_TERMS; ++t) kt[t] = block_sum(kt[t], sh);
    }
    const double kin = kt[0], live = kt[1];
    if (threadIdx.x == 0) {
        double *row = ar.ring + (S.ring0 + step % S.ring_cap) * NDIAG;
        R E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
        if (vertex_valid(S, S.probe[0], S.probe[1], S.probe[2])) {
            const FieldPtrs<R> f = field_ptrs<R>(S, ar, step % 3, (step + 1) % 3, (int)(step % 3));
            vertex_EB<R>(S, f, S.probe[0], S.probe[1], S.probe[2], E, B);
        }
        const int *offn = ar.offs[(step + 1) & 1];
        const long long g = S.key0 + S.nkeys;
        row[0] = (double)step;
        row[1] = ((double)step + 0.5) * S.dt;
        row[2] = mesh ? q * S.dV : 0.0;
        row[3] = mesh ? (rmax > 0.0 ? res / rmax : 0.0) : 0.0;
        row[4] = pw * S.dxdy_mu0;
        row[5] = mesh ? wf * S.dV : 0.0;
        row[6] = mesh ? kin * S.mc2 : 0.0;
        for (int a = 0; a < 3; ++a) {
            row[7 + a] = (double)E[a];
            row[10 + a] = (double)B[a];
        }
        row[13] = (double)(offn[g + 1] - offn[g]);
        int nf = ar.flags[blockIdx.x] ? 1 : 0;
        for (int a = 2; a < 13; ++a)
            if (!isfinite(row[a])) nf = 1;
        if (nf) atomicOr(&ar.flags[blockIdx.x], 2);
        row[14] = (double)nf;
        row[15] = mesh ? 1.0 : 0.0;
        for (int h = 0; h < 3; ++h)
            row[16 + h] = mesh && live > 0.0
                              ? sqrt(kt[2 + 2 * h] * kt[2 + 2 * h] + kt[3 + 2 * h] * kt[3 + 2 * h]) / live
                              : 0.0;
        row[19] = 0.0;
        for (int h = 0; h < 3; ++h) row[20 + h] = 0.0;  // the spectrum's first three, below
        row[23] = 0.0;
        for (int p = 0; p < 3; ++p) row[24 + p] = p < S.n_extra ? px[p] * S.dxdy_mu0 : 0.0;
        row[27] = pt[1] * S.dxdy_mu0;
        row[28] = S.zu0 + S.zu_rate * row[1];
    }
    if (S.spec_on) {
        // mean power at each frequency since the spectrum started, T = (number
        // of samples) dt, in the bunch frame and in the lab
        const double T = ((double)(step + 1 - S.step0)) * S.dt;
        const double k = T > 0.0 ? 2.0 / (T * T) * S.dxdy_mu0 : 0.0;
        double *sr = ar.srow + S.srow0 + (step % S.ring_cap) * 2 * S.nfreq;
        double *row = ar.ring + (S.ring0 + step % S.ring_cap) * NDIAG;
        for (int fq = 0; fq < S.nfreq; ++fq) {  // uniform over the block
            double vr = 0.0, vl = 0.0;
            for (int b = threadIdx.x; b < S.nb_plane; b += BLOCK) {
                const double *o = ar.partial + S.part_plane0 + (long long)PLANE_STRIDE * b;
                vr += o[2 + 2 * fq];
                vl += o[3 + 2 * fq];
            }
            vr = block_sum(vr, sh);
            vl = block_sum(vl, sh);
            if (threadIdx.x == 0) {
                sr[fq] = k * vr;
                sr[S.nfreq + fq] = k * vl;
                if (fq < 3) row[20 + fq] = k * vr;
            }
        }
    }
    if (threadIdx.x == 0) {
        // every block has read the step counter before it counts itself done
        if (atomicAdd(ar.fin_ctr, 1) == (int)gridDim.x - 1) {
            *ar.fin_ctr = 0;
            *ar.d_step = step + 1;
        }
    }
}

// E and B at every vertex of one simulation for the last completed push
// (levels s-1 and s after s steps), in double, component-major.
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_vertex_fields(const SimDev *__restrict__ sims, int sim,
                                                          long long g0, long long count, Arena ar,
                                                          double *__restrict__ out)
{
    const SimDev &S = sims[sim];
    const long long step = *ar.d_step;
    const long long e = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (e >= count) return;
    const long long g = g0 + e;
    const int i = (int)(g % S.n[0]), j = (int)((g / S.n[0]) % S.n[1]),
              k = (int)(g / ((long long)S.n[0] * S.n[1]));
    R E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
    if (step > 0 && vertex_valid(S, i, j, k)) {
        const FieldPtrs<R> f = field_ptrs<R>(S, ar, (step + 2) % 3, step % 3, (int)((step + 2) % 3));
        vertex_EB<R>(S, f, i, j, k, E, B);
    }
    for (int a = 0; a < 3; ++a) {
        out[a * count + e] = (double)E[a];
        out[(3 + a) * count + e] = (double)B[a];
    }
}

// count values of a mesh array, widened to double
__global__ __launch_bounds__(BLOCK) void k_to_double(const float *__restrict__ src, long long count,
                                                      double *__restrict__ out)
{
    const long long e = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (e < count) out[e] = (double)src[e];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define MITHRA_STENCIL_SHAPES(X) \
    X(64, 4) X(32, 8) X(128, 2) X(64, 2) X(32, 4) X(16, 16) X(256, 1) X(128, 1) X(128, 4) X(256, 2) X(64, 8)

bool stencil_shape_supported(int tx, int ty)
{
#define CHECK(a, b) if (tx == a && ty == b) return true;
    MITHRA_STENCIL_SHAPES(CHECK)
#undef CHECK
    return false;
}

template <typename R>
void launch_stencil(hipStream_t st, const SimDev *sims, const int4 *items, int nitems,
                    const Arena &ar, int tx, int ty, int kz, int fuse_x)
{
    if (nitems <= 0) return;
    dim3 grid(nitems, 4);
#define LAUNCH(a, b)                                                                        \
    if (tx == a && ty == b) {                                                               \
        hipLaunchKernelGGL((k_stencil<R, a, b>), grid, dim3(a * b), 0, st, sims, items, ar, \
                           kz, fuse_x);                                                     \
        return;                                                                             \
    }
    MITHRA_STENCIL_SHAPES(LAUNCH)
#undef LAUNCH
}

template <typename R>
void launch_boundary(hipStream_t st, const SimDev *sims, const BSeg *segs, int nseg,
                     long long total, const Arena &ar)
{
    if (total <= 0) return;
    long long nb = (total + BLOCK - 1) / BLOCK;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL((k_boundary<R>), dim3((unsigned)nb), dim3(BLOCK), 0, st, sims, segs, nseg,
                       total, ar);
}

template <typename R>
void launch_mur2(hipStream_t st, const SimDev *sims, const BSeg *segs, int nseg, long long total,
                 const Arena &ar)
{
    if (total <= 0) return;
    long long nb = (total + BLOCK - 1) / BLOCK;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL((k_mur2<R>), dim3((unsigned)nb), dim3(BLOCK), 0, st, sims, segs, nseg, total,
                       ar);
}

// whole rounds of 8 bricks
static int dealt_grid(int nbricks, int4 bs)
{
    return (int)((nbricks + 7) / 8 * 8LL * bs.w);
}

template <typename R>
void launch_push(hipStream_t st, const SimDev *sims, const Brick *bricks, int nbricks, int4 bs,
                 const Arena &ar, int optical)
{
    if (nbricks <= 0) return;
    if (optical)
        hipLaunchKernelGGL((k_push<R, true>), dim3(dealt_grid(nbricks, bs)), dim3(BLOCK), 0, st,
                           sims, bricks, nbricks, bs, ar);
    else
        hipLaunchKernelGGL((k_push<R, false>), dim3(dealt_grid(nbricks, bs)), dim3(BLOCK), 0, st,
                           sims, bricks, nbricks, bs, ar);
}

template <typename R>
void launch_deposit(hipStream_t st, const SimDev *sims, const Brick *bricks, int nbricks, int4 bs,
                    const Arena &ar, int init)
{
    if (nbricks <= 0) return;
    hipLaunchKernelGGL((k_deposit<R>), dim3(dealt_grid(nbricks, bs)), dim3(BLOCK), 0, st, sims,
                       bricks, nbricks, bs, ar, init);
}

void launch_scan(hipStream_t st, const Arena &ar, long long nkeys_total, int *block_sums,
                 int nblocks, const int4 *chunks)
{
    hipLaunchKernelGGL(k_scan_reduce, dim3(nblocks), dim3(BLOCK), 0, st, ar.counts, nkeys_total,
                       block_sums, chunks, ar);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, st, block_sums, nblocks);
    hipLaunchKernelGGL(k_scan_down, dim3(nblocks), dim3(BLOCK), 0, st, ar.counts, nkeys_total,
                       block_sums, chunks, ar);
}

template <typename R>
void launch_scatter(hipStream_t st, const Arena &ar, long long np)
{
    if (np <= 0) return;
    hipLaunchKernelGGL((k_scatter<R>), dim3((unsigned)((np + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                       st, ar, np);
}

template <typename R>
void launch_diag(hipStream_t st, const SimDev *sims, int nsim, const int2 *plane_items,
                 int nplane, const int2 *mesh_items, int nmesh, const int2 *kin_items, int nkin,
                 const Arena &ar)
{
    const int nparts = nplane + nmesh + nkin;
    if (nparts > 0)
        hipLaunchKernelGGL((k_diag_parts<R>), dim3(nparts), dim3(BLOCK), 0, st, sims, plane_items,
                           nplane, mesh_items, nmesh, kin_items, ar);
    hipLaunchKernelGGL((k_diag_final<R>), dim3(nsim), dim3(BLOCK), 0, st, sims, ar);
}

void launch_seed_beam(hipStream_t st, const SimDev *sims, int sim, int ncol,
                      const long long *d_step)
{
    hipLaunchKernelGGL(k_seed_beam, dim3((unsigned)((2 * ncol + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                       st, sims, sim, ncol, d_step);
}

template <typename R>
void launch_background(hipStream_t st, const SimDev *sims, int sim, long long ncell,
                       const Arena &ar)
{
    hipLaunchKernelGGL((k_background<R>), dim3((unsigned)((ncell + BLOCK - 1) / BLOCK)),
                       dim3(BLOCK), 0, st, sims, sim, ncell, ar);
}

template <typename R>
void launch_vertex_fields(hipStream_t st, const SimDev *sims, int sim, long long g0,
                          long long count, const Arena &ar, double *out6)
{
    hipLaunchKernelGGL((k_vertex_fields<R>), dim3((unsigned)((count + BLOCK - 1) / BLOCK)),
                       dim3(BLOCK), 0, st, sims, sim, g0, count, ar, out6);
}

void launch_to_double(hipStream_t st, const float *src, long long count, double *out)
{
    hipLaunchKernelGGL(k_to_double, dim3((unsigned)((count + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                       st, src, count, out);
}

#define MITHRA_INSTANTIATE(R)                                                                   \
    template void launch_stencil<R>(hipStream_t, const SimDev *, const int4 *, int,             \
                                    const Arena &, int, int, int, int);                         \
    template void launch_boundary<R>(hipStream_t, const SimDev *, const BSeg *, int, long long, \
                                     const Arena &);                                            \
    template void launch_mur2<R>(hipStream_t, const SimDev *, const BSeg *, int, long long,     \
                                 const Arena &);                                                \
    template void launch_push<R>(hipStream_t, const SimDev *, const Brick *, int, int4,         \
                                 const Arena &, int);                                           \
    template void launch_deposit<R>(hipStream_t, const SimDev *, const Brick *, int, int4,      \
                                    const Arena &, int);                                        \
    template void launch_scatter<R>(hipStream_t, const Arena &, long long);                     \
    template void launch_diag<R>(hipStream_t, const SimDev *, int, const int2 *, int,           \
                                 const int2 *, int, const int2 *, int, const Arena &);          \
    template void launch_vertex_fields<R>(hipStream_t, const SimDev *, int, long long,          \
                                          long long, const Arena &, double *);                  \
    template void launch_background<R>(hipStream_t, const SimDev *, int, long long,             \
                                       const Arena &);

MITHRA_INSTANTIATE(float)
MITHRA_INSTANTIATE(double)

}  // namespace mithra

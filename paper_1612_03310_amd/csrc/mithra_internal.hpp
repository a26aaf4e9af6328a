// Internal types shared by the kernels and the runtime of the MI355X path.
// Not part of the public ABI (see include/mithra.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mithra {

// Particles are binned by cell in tiles of 8x8x8 cells; a cell's bin key is
// tile * 512 + (lz * 8 + ly) * 8 + lx (tile-major, x fastest inside the tile),
// so one tile's particles and one row of cells inside a tile are contiguous.
constexpr int TILE = 8;
constexpr int TILE_CELLS = TILE * TILE * TILE;
constexpr int TILE_VERT = TILE + 1;  // vertices per axis a tile's cells touch
constexpr int NKINDS = 7;            // kernel kinds for timing
constexpr int NDIAG = 29;            // doubles per diagnostic row
constexpr int BLOCK = 256;
constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_CHUNK = BLOCK * SCAN_PER_THREAD;
constexpr int MESH_DIAG_PER_THREAD = 8;
constexpr int KIN_PER_THREAD = 8;
constexpr int MAXF = 32;            // normalized frequencies of the plane spectrum
constexpr int SPEC_PER_FREQ = 8;    // per power-plane point and frequency: (Ex, Ey, Bx, By) x (re, im)
constexpr int PLANE_STRIDE = 2 + 2 * MAXF;  // per plane block: power, lab power, and per
                                             // frequency the bunch-frame and lab terms
constexpr int KIN_TERMS = 8;         // per kinetic block: sum (gamma - 1), live count,
                                     // cos and sin sums of h K z for h = 1, 2, 3
constexpr int OKEY_LOST = 1 << 9;

enum Kind { K_STENCIL = 0, K_BOUNDARY, K_PUSH, K_DEPOSIT, K_SCAN, K_SCATTER, K_DIAG };

// Per-simulation constants, read by every kernel (device copy in an array).
struct SimDev {
    int n[3];
    int bc[3];          // 1: periodic axis, 0: absorbing (Mur) faces
    int mur2;           // the Mur faces are of second order
    int sc;             // space charge on
    int nsub;           // particle sub-steps per field step
    int nt[3];          // tiles per axis
    int nkeys;          // nt0*nt1*nt2*512; key nkeys is the "lost" bucket
    int np;             // particles of this simulation (live + lost)
    long long cell0;    // offset of this simulation in the mesh arenas
    long long key0;     // offset in the key arenas (nkeys + 1 entries)
    long long part0;    // offset in the particle arenas
    int tile0;          // offset in the per-tile arrays
    // diagnostics
    int probe[3];
    int kp;
    int mesh_every;     // 0: never
    int ring_cap;
    long long ring0;    // first row of this simulation in the ring arena
    int part_plane0, nb_plane;  // partial-sum slots
    int kp_extra[3], n_extra;   // further sampling plates (power only), how many
    int part_extra0;            // their partial-sum slots, nb_plane per plate
    int part_mesh0, nb_mesh;
    int part_kin0, nb_kin;
    // potential update, eq. (updateEquation) in the regrouped form
    double a1, ax, ay, az, A, srcA, srcPhi;
    double murb0[3], murb1[3];  // first-order Mur beta_0 (= beta_4), beta_1 (= beta_3)
    double murg[3][4];  // second-order Mur, per face axis: gamma_0 (= gamma_4),
                        // gamma_1 (= gamma_3), and the transverse weights along
                        // the lower (gamma_5,6,9,10) and higher (7,8,11,12) other axis
    // vertex fields
    double inv_dt, inv_2d[3];
    // particles
    double d[3], origin[3];
    double kE;          // q dtb / (2 m c): E [V/m] -> half kick of u
    double kB;          // q dtb / (2 m):   B [T] * kB / gamma = Boris rotation vector
    double cdtb_d[3];   // c dtb / d_a
    double dt, dtb;
    // undulator in the rest frame
    double ku, kz_cell, phase_off, phase_rate;
    double EuK, BuyK, BuzK;  // kick-scaled amplitudes of E_x, B_y, B_z
    // deposition: rho and J per unit of particle weight
    double rho_unit, J_unit[3];
    // diagnostics (SI)
    double dV, mc2, dxdy_mu0, eps0_half, inv_2mu0;
    double kbunch;      // 2 gamma0 k_u: wave number of the bunching factor
    double omega1;      // gamma0 beta0 c k_u: rest-frame resonant frequency
    long long spec0;    // first double of this simulation in the plane-spectrum arena
    int spec_on;        // the plane spectrum is sampled
    int nfreq;          // normalized frequencies of the spectrum, fnu[f] = omega_f / omega1
    double fnu[MAXF];
    long long step0;    // step at which the spectrum (re)started
    long long srow0;    // first double of this simulation in the spectrum-row arena
    // FEL output in the lab: fields of the bunch frame seen in the lab
    // (gamma0, gamma0 beta0), and the power plane's lab undulator position
    // z' = zu0 + zu_rate t
    double lab_g, lab_gb, zu0, zu_rate;
    double und_kL;      // k_u L of a finite undulator (exit at z' = L), 0: unbounded
    // seed plane wave along +z (TF/SF planes k = 2 and 3)
    int seed_on, seed_sig;
    double seed_a0, seed_p[2], seed_f, seed_t0, seed_tau, seed_cep, seed_zref;
    // its beam: 0 plane wave (uniform corrections), 1 Gaussian beam along +z,
    // whose per-column corrections of A_x and A_y on planes 2 and 3 are
    // written each step to seed_corr ([comp][plane][ny][nx])
    int seed_beam;
    double seed_zr[2], seed_focus[3], seed_k;
    double *seed_corr;
    // static background charge density at the vertices (R, this simulation's
    // cells) and the sum rho + background the potential update of phi reads
    // (written before it each step); both null when there is none
    void *bg, *rho_bg;
    // optical undulator: a plane wave towards -z, A = a p s(t + (z - z_ref)/c),
    // in place of the static undulator (same signal shapes as the seed)
    int opt_on, opt_sig;
    double opt_a, opt_p[2], opt_f, opt_t0, opt_tau, opt_cep, opt_zref;
    // its beam: 0 plane wave, 1 Gaussian beam (Rayleigh lengths along p and
    // along z x p, focus, carrier wave number 2 pi f / c)
    int opt_beam;
    double opt_zr[2], opt_focus[3], opt_k;
};

// Device buffers of a batch (one arena per quantity, simulations concatenated).
struct Arena {
    void *pot[3][4];    // potential levels (rotating mod 3) x {Ax, Ay, Az, phi}
    void *J[3];
    void *rho[2];       // rho^{s+1/2} in rho[s & 1]
    int *counts;        // per key (all simulations), zero between steps
    int *offs[2];       // bucket starts; offs[s & 1] describes particle buffer s & 1
    int *key[2];
    void *off[2][3];    // position inside the cell, [0, 1)
    void *u[2][3];
    int *id[2];
    int *okey;          // start of the step, for the deposit: x inside the tile (3 bits)
                        // and the cell move per axis (2 bits each, move + 1), or
                        // OKEY_LOST for a particle lost in the step
    void *ooff[3];
    double *ke;         // (gamma - 1) by particle id, for the kinetic-energy sum
    double *zr;         // rest-frame z by particle id (NaN once lost), for the bunching factor
    double *partial;    // diagnostic partial sums
    double *spec;       // running DFT of the power-plane fields at the frequencies, per simulation
                        // sum-major: sum q = 8 f + c of plane point e at spec0 + q * nx * ny + e
                        // (reset at commit)
    double *srow;       // per diagnostic row: the mean power at each frequency, bunch frame
                        // then lab (2 nfreq doubles at srow0 + (step % ring_cap) * 2 nfreq)
    double *ring;       // diagnostic rows
    int *flags;         // per simulation: a non-finite value was produced
    int *tact;          // per tile: a particle in the 27-tile neighbourhood at the start of
                        // the step (set by the push, cleared by the deposit)
    int *pocc[2];       // per tile: particles may sit in it at the start of step s
                        // (pocc[s & 1]; written by the push of step s - 1)
    int *jdirty;        // per tile: J holds non-zero values
    int *rdirty[2];     // per tile: rho[b] holds non-zero values
    long long *d_step;  // completed steps (all simulations advance together); the
                        // diagnostics advance it at the end of a step
    int *fin_ctr;       // row-writing blocks done in this step (back to 0 after it)
};

// The push and the deposit deal tiles to the XCDs in bricks of bx x by x bz
// tiles (the brick shape, chosen by the tuner): the brick table lists, per
// simulation, the bricks of its tile grid in order, x fastest.
struct Brick {
    int sim;   // simulation
    int g0;    // global index of the brick's first tile
    int t0[3]; // its first tile, in tile coordinates
    int nt[3]; // the simulation's tiles per axis
};

struct BSeg {
    int sim, comp, group, pad;  // group: axis of the faces
    long long start, count;
};

// Host-side launchers (kernels.hip).
template <typename R>
// fuse_x: the stencil pass also updates the x faces (first-order Mur)
void launch_stencil(hipStream_t st, const SimDev *sims, const int4 *items, int nitems,
                    const Arena &ar, int tx, int ty, int kz, int fuse_x);
// Gaussian-beam seed: the TF/SF corrections of simulation `sim` for this
// step (ncol = nx * ny columns), before its potential update
void launch_seed_beam(hipStream_t st, const SimDev *sims, int sim, int ncol,
                      const long long *d_step);
// background charge: rho + background of simulation `sim` for this step
template <typename R>
void launch_background(hipStream_t st, const SimDev *sims, int sim, long long ncell,
                       const Arena &ar);
template <typename R>
void launch_boundary(hipStream_t st, const SimDev *sims, const BSeg *segs, int nseg,
                     long long total, const Arena &ar);
// second-order Mur, one stage (faces, edges or corners) per call
template <typename R>
void launch_mur2(hipStream_t st, const SimDev *sims, const BSeg *segs, int nseg, long long total,
                 const Arena &ar);
// push and deposit: bricks of bs.x x bs.y x bs.z tiles (bs.w tiles a brick)
// dealt to the XCDs; optical: some simulation has the optical undulator on
template <typename R>
void launch_push(hipStream_t st, const SimDev *sims, const Brick *bricks, int nbricks, int4 bs,
                 const Arena &ar, int optical);
template <typename R>
void launch_deposit(hipStream_t st, const SimDev *sims, const Brick *bricks, int nbricks, int4 bs,
                    const Arena &ar, int init);
// chunks: per chunk of SCAN_CHUNK keys, (first global tile, last global tile,
// holds a lost bucket), for skipping chunks of unoccupied tiles
void launch_scan(hipStream_t st, const Arena &ar, long long nkeys_total, int *block_sums,
                 int nblocks, const int4 *chunks);
template <typename R>
void launch_scatter(hipStream_t st, const Arena &ar, long long nparticles);
template <typename R>
void launch_diag(hipStream_t st, const SimDev *sims, int nsim, const int2 *plane_items,
                 int nplane, const int2 *mesh_items, int nmesh, const int2 *kin_items, int nkin,
                 const Arena &ar);
// E and B of cells g0 .. g0+count-1 of simulation `sim` into out6: component
// a (Ex, Ey, Ez, Bx, By, Bz) of cell g0 + e at out6[a * count + e]
// E and B of cells g0 .. g0+count-1 of simulation `sim` into out6: component
// a (Ex, Ey, Ez, Bx, By, Bz) of cell g0 + e at out6[a * count + e]
template <typename R>
void launch_vertex_fields(hipStream_t st, const SimDev *sims, int sim, long long g0,
                          long long count, const Arena &ar, double *out6);
void launch_to_double(hipStream_t st, const float *src, long long count, double *out);
bool stencil_shape_supported(int tx, int ty);

}  // namespace mithra

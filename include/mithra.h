/*
 * mithra.h -- C ABI of the MI355X (gfx950) implementation of the per-step
 * particle-in-cell loop of MITHRA's full-wave FEL method (Fallahi, Yahaghi,
 * Kaertner, arXiv:1612.03310), solved in the bunch rest frame:
 *
 *   1. potential update, eq. (updateEquation) (NSFD, eq. (NSFDtrick)),
 *      for A_x, A_y, A_z and phi, with first-order Mur boundaries
 *      (section "Boundary Truncation", first-order ABCs);
 *   2. E and B at the cell vertices from the potentials (section "Field
 *      Evaluation"), linear interpolation to each macro-particle
 *      (eq. (fieldInterpolation)), plus the undulator field seen in the rest
 *      frame (eqs. (undulatorField), (undulatorFieldRest), fringe field);
 *   3. Boris push (eq. (BorisScheme)) with N sub-steps per field step;
 *   4. charge and current deposition (section "Current Deposition",
 *      eq. (currentIntegral)), charge-conserving;
 *   5. double-precision diagnostics (charge, continuity, radiated power,
 *      energies, field probe, bunching factor, power at the harmonics).
 *
 * Also: second-order Mur boundaries; a seed brought in through the
 * total-field/scattered-field planes and an optical undulator, each a plane
 * wave or a Gaussian beam; a static background charge (test fixture);
 * checkpoints; batches of independent simulations replayed from one
 * captured HIP graph, with a tile autotuner.
 *
 * Conventions used by every call:
 *   - SI units in and out; the rest frame of the bunch (the frame moving with
 *     beta0 = sqrt(1 - 1/gamma0^2), gamma0 = gamma / sqrt(1 + K^2/2),
 *     section "Lorentz Transformation").
 *   - Mesh arrays hold n[0]*n[1]*n[2] values, x fastest: element
 *     (k*n[1] + j)*n[0] + i is grid point (i, j, k).  phi and rho sit on the
 *     vertices origin + (i dx, j dy, k dz); A_l and J_l on the l-edges
 *     (A_x at i+1/2, A_y at j+1/2, A_z at k+1/2).  Along its own axis an edge
 *     grid has n-1 points on a Mur axis, so its last array layer is unused
 *     and reads as zero.
 *   - Time levels: after s completed steps the newest potentials are A^s,
 *     phi^s (phi^s belongs to t = (s+1/2) dt, section "FDTD for Scalar
 *     Potential"); particle positions belong to t = (s+1/2) dt and momenta
 *     u = gamma*beta half a particle sub-step earlier (t = s dt with one
 *     sub-step).  Input particles are taken at s = 0; the potentials start
 *     at zero and J^0 = 0.
 *   - Every call returns a mithra_status; nothing throws across the ABI.
 *     On error mithra_last_error() gives a message naming the violated
 *     condition (a thread-local string, valid until the next call on the
 *     same thread).
 *   - Host arrays belong to the caller.  The library copies them in and out
 *     synchronously on the simulation's stream.  The library owns all device
 *     memory of a simulation and frees it in mithra_destroy.
 *   - A simulation and its stream must not be used from two threads at once.
 */
#ifndef MITHRA_H
#define MITHRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mithra_sim mithra_sim;
typedef struct mithra_batch mithra_batch;

typedef enum {
    MITHRA_OK = 0,
    MITHRA_EINVAL = 1,   /* argument out of range, unstable mesh, bad size */
    MITHRA_ENOMEM = 2,   /* device or host allocation failed */
    MITHRA_EDEVICE = 3,  /* HIP runtime error, no gfx950 device */
    MITHRA_ENUMERIC = 4, /* a non-finite momentum or diagnostic was produced */
    MITHRA_ESTATE = 5    /* call not valid in the current state */
} mithra_status;

typedef enum {
    MITHRA_F64 = 0,      /* fields, push and positions in double precision */
    MITHRA_F32_SPLIT = 1 /* fields and push in float, positions as int32 cell
                            + float offset, diagnostics in double */
} mithra_precision;

typedef enum {
    MITHRA_BC_MUR1 = 0,     /* first-order Mur absorbing boundary (section
                               "Boundary Truncation", beta coefficients) */
    MITHRA_BC_PERIODIC = 1, /* wrap-around (test configurations) */
    MITHRA_BC_MUR2 = 2      /* second-order Mur (same section): faces by the
                               printed gamma_0..12 update, edges and corners
                               from the face conditions involved, added at
                               the centre of the edge square or corner cube.
                               The absorbing axes of one mesh share one order
                               (mixing 0 and 2 is EINVAL). */
} mithra_bc;

typedef enum {
    MITHRA_AX = 0, MITHRA_AY = 1, MITHRA_AZ = 2, MITHRA_PHI = 3, /* newest level */
    MITHRA_JX = 4, MITHRA_JY = 5, MITHRA_JZ = 6,                 /* J^s */
    MITHRA_RHO = 7,                                              /* rho^{s+1/2} */
    MITHRA_EX = 8, MITHRA_EY = 9, MITHRA_EZ = 10,                /* self field used by */
    MITHRA_BX = 11, MITHRA_BY = 12, MITHRA_BZ = 13,              /* the last push */
    MITHRA_AX_PREV = 14, MITHRA_AY_PREV = 15, MITHRA_AZ_PREV = 16,
    MITHRA_PHI_PREV = 17,                                        /* level s-1 */
    MITHRA_RHO_PREV = 18                                         /* rho^{s-1/2} */
} mithra_field;

/* MESH: the computational box in the rest frame (job-file section MESH). */
typedef struct {
    int32_t n[3];       /* grid points per axis, each >= 8 */
    double d[3];        /* dx, dy, dz [m], > 0 */
    double origin[3];   /* position of grid point (0,0,0) [m]; the undulator
                           axis is x = y = 0 */
    double courant;     /* nu = c dt / dz, in (0, 1] (dt = dz / c is nu = 1) */
    double nsfd_A;      /* NSFD weight A of eq. (NSFDtrick); < 0 selects
                           eq. (NSFDCoefficient) */
    int32_t substeps;   /* N = dt / dt_b >= 1 particle sub-steps per field step */
    int32_t space_charge; /* 0: phi == 0; 1: phi from eq. (HelmholtzF) */
    int32_t bc[3];      /* mithra_bc per axis (both faces of the axis) */
} mithra_mesh;

/* Seed (section "Seed Field"): a plane wave of vector potential travelling
   towards +z in the rest frame,
     A(z, t) = amplitude (polarization[0], polarization[1], 0) s(t - (z - z_ref)/c),
   brought into the mesh by the total-field/scattered-field technique: after
   each update the scattered-field plane k = 2 loses, and the total-field
   plane k = 3 gains, the incident field its update took from, or missed on,
   the other plane.  Everything from plane 3 on carries the seed.  s is one
   of the printed signal shapes (section "FIELD", field-initialization) with
   x = t - t0:
     NEUMANN   -4 ln2 cos(2 pi f x + cep) x / tau^2 exp(-2 ln2 x^2 / tau^2)
     GAUSSIAN  cos(2 pi f x + cep) exp(-2 ln2 x^2 / tau^2)
     SECANT    cos(2 pi f x + cep) / cosh(x / tau)
     FLAT_TOP  the Gaussian for x <= 0, then the bare carrier (the printed
               "sinusoidal pulse"). */
typedef enum {
    MITHRA_SIGNAL_NEUMANN = 0,
    MITHRA_SIGNAL_GAUSSIAN = 1,
    MITHRA_SIGNAL_SECANT = 2,
    MITHRA_SIGNAL_FLAT_TOP = 3
} mithra_signal;

typedef struct {
    double amplitude;       /* A0 [V s / m]; 0 switches the seed off */
    double polarization[2]; /* x and y weights of the polarization (used as given) */
    double frequency;       /* carrier frequency f [Hz], rest frame, >= 0 */
    double t0;              /* signal centre [s] */
    double tau;             /* signal width [s], > 0 */
    double cep;             /* carrier-envelope phase [rad] */
    double z_ref;           /* position where the wave reads s(t) [m] */
    int32_t signal;         /* mithra_signal */
    int32_t pad;
} mithra_seed;

/* UNDULATOR: static planar undulator, eq. (undulatorField), and the beam
   energy that fixes the frame. */
typedef struct {
    double lambda_u;    /* lab period [m] > 0 */
    double K;           /* undulator parameter >= 0; B0 = 2 pi m c K / (e lambda_u) */
    double gamma_beam;  /* lab mean Lorentz factor; gamma0 = gamma / sqrt(1 + K^2/2) > 1 */
    double z_entrance;  /* rest-frame z of the lab entrance z' = 0 at t = 0 [m];
                           z' = gamma0 (z - z_entrance + beta0 c t) */
    double length;      /* total lab length L [m] (section "UNDULATOR", length), a whole
                           number of periods (else EINVAL); past the exit z' = L the field
                           is the entrance fringe mirrored about L, so a particle that
                           crosses the whole undulator keeps no transverse kick.
                           <= 0: unbounded */
} mithra_undulator;

typedef struct {
    int32_t probe[3];        /* vertex of the field probe */
    int32_t power_plane_k;   /* z index of the plane of the power diagnostic */
    int32_t mesh_diag_every; /* mesh-wide terms every M steps (M >= 1), 0 = never */
    int32_t capacity;        /* rows kept in the device ring (>= 1) */
    int32_t power_spectrum;  /* 1: sample the running DFT of the power plane each step for
                                mithra_diag_row.power_harmonic (FEL output); 0 (default):
                                off, power_harmonic = 0.  Changes only before the first step */
    int32_t extra_planes[3]; /* z indices of further sampling plates (section "FEL-OUTPUT":
                                the plate distance may be repeated), -1 for none: the
                                radiated power through each, mithra_diag_row.power_extra */
} mithra_diag_cfg;

/* One row per completed step s (fields at t = (s+1/2) dt). */
typedef struct {
    int64_t step;
    double t;
    double total_charge;        /* sum rho^{s+3/2} dV [C]                   (mesh term) */
    double continuity_residual; /* max|rho^{s+3/2} - rho^{s+1/2} + dt div J^{s+1}|
                                   / max|rho^{s+3/2}|                      (mesh term) */
    double power;               /* sum (Ex By - Ey Bx) / mu0 dx dy over plane k [W] */
    double field_energy;        /* sum (eps0 E^2/2 + B^2/(2 mu0)) dV [J]     (mesh term) */
    double kinetic_energy;      /* sum (gamma - 1) m c^2 over live particles (mesh term) */
    double probe_E[3], probe_B[3];
    int64_t lost;               /* particles lost so far */
    int32_t nonfinite;          /* a non-finite value was produced */
    int32_t has_mesh_terms;     /* 1 if the mesh terms were computed this step */
    double bunching[3];         /* |<exp(i h K z)>| over live particles, h = 1, 2, 3, after
                                   the push; z the rest-frame longitudinal position,
                                   K = 2 gamma0 k_u the ponderomotive wave number in
                                   this frame (section "Bunching factor")  (mesh term) */
    double power_harmonic[3];   /* (with power_spectrum on) mean power [W] carried through
                                   plane k at the first three normalized frequencies of
                                   mithra_set_spectrum (default nu omega_1 for nu = 1, 2, 3,
                                   omega_1 = gamma0 beta0 c k_u the rest-frame resonant
                                   frequency), since the spectrum started (the last
                                   particle load): (2/T^2) sum Re(F_Ex F_By* - F_Ey F_Bx*)/mu0
                                   dx dy with F(omega) = sum_n f(t_n) exp(-i omega t_n) dt the
                                   running DFT of the plane's vertex fields and T = (number of
                                   samples) dt; 0 beyond the number of frequencies */
    double power_extra[3];      /* radiated power [W] through the further plates of
                                   mithra_diag_cfg.extra_planes, as power; 0 where none */
    double power_lab;           /* FEL output in the lab (section "FEL-OUTPUT"): the flux of
                                   the lab Poynting vector of the self field through plane k,
                                   the plane's fields seen in the lab (frame moving along +z at
                                   beta0 c): E_x' = g (E_x + b c B_y), E_y' = g (E_y - b c B_x),
                                   B_x' = g (B_x - b E_y / c), B_y' = g (B_y + b E_x / c),
                                   g = gamma0, b = beta0; (E_x' B_y' - E_y' B_x')/mu0 dx dy [W].
                                   A forward plane wave gives gamma0^2 (1 + beta0)^2 power */
    double z_undulator;         /* the lab undulator position of plane k at this row's time,
                                   z' = gamma0 (z_k - z_entrance + beta0 c t) [m]: the abscissa
                                   of the FEL output (power against undulator position) */
} mithra_diag_row;

/* Derived constants and bookkeeping of a simulation. */
typedef struct {
    double dt, dtb;           /* field and particle time step [s] */
    double nsfd_A;            /* NSFD weight in use */
    double gamma0, beta0;     /* frame of the undulator-averaged bunch */
    double B0, ku;            /* undulator peak field [T] and wave number [1/m] */
    int64_t step;             /* completed steps */
    int64_t np;               /* particles loaded (live + lost) */
    int64_t device_bytes;     /* device memory held */
    int32_t stencil_tile[3];  /* x, y columns per block and z planes per block */
    int32_t precision;        /* mithra_precision */
    int32_t particle_brick[3]; /* tiles of 8^3 cells per brick along x, y, z: the push and the
                                  deposit deal bricks of tiles to the XCDs (from the tuner) */
    int32_t pad;
} mithra_info;

/* ---- single simulation -------------------------------------------------- */

/* Create a simulation.  Validates the mesh (the stability condition of the
   NSFD scheme, section "Numerical Dispersion in FDTD": the largest value of
   the right-hand side of eq. (NSFDDispersionCD) over the Brillouin zone must
   not exceed 1) instead of adapting it; EINVAL names the violated condition.
   stream: a hipStream_t; NULL makes the simulation create and own a
   non-blocking stream (graph capture needs a stream other than the legacy
   default stream).  EDEVICE if the current device is not gfx950. */
mithra_status mithra_create(const mithra_mesh *mesh, const mithra_undulator *und,
                            mithra_precision prec, void *stream, mithra_sim **out);

/* Route device allocations through alloc(bytes, ctx) / release(ptr, ctx)
   (e.g. a PyTorch caching allocator) for simulations created afterwards.
   NULL functions restore hipMalloc/hipFree. */
mithra_status mithra_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                                   void (*release)(void *ptr, void *ctx), void *ctx);

/* Load np macro-particles (section "Electron Bunch Generation" produces them;
   the caller supplies the result).  pos: [np][3] rest-frame positions [m] at
   t = (s+1/2) dt; u: [np][3] gamma*beta half a particle sub-step earlier, at
   t = (s+1/2) dt - dtb/2 (= s dt with one sub-step); q_macro, m_macro: charge
   [C] (signed) and mass [kg] of one macro-particle.  Particles whose cell is
   outside [2, n-3] on an axis are counted as lost at once.  Deposits
   rho^{s+1/2}; sets J^s = 0.  EINVAL for np < 0, non-finite input, m <= 0
   or more than 2^31 - 2^20 particles (32-bit bucket offsets; in a batch the
   limit holds for all simulations together). */
mithra_status mithra_set_particles(mithra_sim *sim, int64_t np, const double *pos,
                                   const double *u, double q_macro, double m_macro);

/* Test fixture: a static background charge density rho_bg [C/m^3] at the
   vertices (n[0]*n[1]*n[2] doubles, x fastest; copied), added to rho in the
   source of phi of eq. (updateEquation) at every step, e.g. the negative of
   the initial bunch charge for a neutral system.  The diagnostics and the
   deposited rho do not include it.  NULL removes it.  EINVAL for a value that
   is not finite; ENOMEM if the two device arrays (the background and
   rho + background) cannot be allocated. */
mithra_status mithra_set_background(mithra_sim *sim, const double *rho_bg);

mithra_status mithra_config_diag(mithra_sim *sim, const mithra_diag_cfg *cfg);

/* Normalized frequencies of the power spectrum (section "FEL-OUTPUT":
   normalized-frequency, repeated, or the sweep from minimum- to
   maximum-normalized-frequency at normalized-frequency-resolution, which the
   caller lists): nu_f = omega_f / omega_1, omega_1 = gamma0 beta0 c k_u the
   rest-frame resonant frequency (a wave along z has the same normalized
   frequency in the lab).  At most MITHRA_MAX_FREQ, each positive; the
   default is 1, 2, 3.  power_harmonic of the rows holds the first three.
   ESTATE after the first step. */
#define MITHRA_MAX_FREQ 32
mithra_status mithra_set_spectrum(mithra_sim *sim, const double *nu, int32_t nfreq);

/* The mean power at each normalized frequency for rows first_step ..
   first_step+count-1 (still in the ring of mithra_diag_cfg.capacity rows):
   rest[r * nfreq + f] in the bunch frame, (2/T^2) sum Re(F_Ex F_By* - F_Ey F_Bx*)
   / mu0 dx dy with the running DFT F of the plane's vertex fields since the
   spectrum started (T its length: from the last particle load or the
   checkpoint's own start), and lab[r * nfreq + f] the same from the DFT of the
   fields seen in the lab (see power_lab).  ESTATE with power_spectrum off;
   EINVAL for rows outside the ring. */
mithra_status mithra_get_spectrum(mithra_sim *sim, int64_t first_step, int64_t count, double *rest,
                                  double *lab);

/* Set (or, with amplitude 0 or seed == NULL, clear) the seed plane wave of
   the simulation; it acts from the next step.  EINVAL for non-finite
   values, tau <= 0, f < 0, an unknown signal, a periodic z axis or fewer
   than 8 planes along z. */
mithra_status mithra_set_seed(mithra_sim *sim, const mithra_seed *seed);

/* Optical undulator (section "UNDULATOR", undulator-type optical, beam-type
   plane wave): replace the static undulator's field acting on the particles
   by a plane wave travelling towards -z, given in the rest frame in the form
   of the seed: A_perp(t, z) = amplitude * polarization * s(t + (z - z_ref)/c),
   s one of the four seed signals, so E = -amplitude * polarization * s',
   B = (-p_y, p_x) * amplitude * s' / c.  The frame (gamma0) stays the one the
   undulator struct of mithra_create defined; give it K = a0 of the wave and
   lambda_u = half the laser wavelength to put the frame on the bunch's mean
   velocity.  Amplitude 0 or wave == NULL switches back to the static
   undulator.  Acts from the next step.  EINVAL for non-finite values,
   tau <= 0, f < 0 or an unknown signal. */
mithra_status mithra_set_optical_undulator(mithra_sim *sim, const mithra_seed *wave);

/* Beam of the optical undulator (section "UNDULATOR": beam types plane wave
   and Gaussian beam, Rayleigh radii parallel and perpendicular to the
   polarization, position = focus).  The paper gives no field; the library's
   reading: the wave above times the paraxial envelope of an astigmatic
   Gaussian beam, A_perp = amplitude * p * Re{U S(t + (z - z_ref)/c)} with S
   the analytic signal (envelope times exp(i(2 pi f x + cep))),
   U = u(xi, z_par) u(eta, z_perp), u(v, z_R) = sqrt(i z_R / q)
   exp(-i k v^2 / (2 q)), q = (z_f - z) + i z_R, k = 2 pi f / c, xi and eta
   the distances from the axis along p/|p| and along z x p/|p|; E = -dA/dt,
   B = curl A (no scalar potential; Gauss's and Ampere's laws then hold to
   the paraxial order 1/(k z_R)).  Waist radius sqrt(2 z_R / k) at the
   focus.  Type 0 is the plane wave (default).  Kept when the wave itself
   changes; acts from the next step.  EINVAL for an unknown type, Rayleigh
   lengths that are not finite and positive, or a focus that is not finite. */
typedef enum { MITHRA_BEAM_PLANE = 0, MITHRA_BEAM_GAUSSIAN = 1 } mithra_beam_type;

typedef struct {
    int32_t type;          /* mithra_beam_type */
    int32_t pad;
    double rayleigh[2];    /* Rayleigh lengths along p and along z x p [m] (Gaussian) */
    double focus[3];       /* focus, rest frame [m] (Gaussian) */
} mithra_beam;

mithra_status mithra_set_optical_beam(mithra_sim *sim, const mithra_beam *beam);

/* Beam of the seed (section "FIELD", seed types plane wave and Gaussian
   beam, same parameters): the seed's wave (mithra_set_seed) times the
   paraxial envelope above for a beam travelling towards +z, with
   zeta = z - z_f in q.  The TF/SF planes then inject, at every point of
   A_x (at x + dx/2) and A_y (at y + dy/2), the incident field of that point,
   and the corrections use each point's own neighbours on the other plane
   (a kernel before each potential update writes them, 4 nx ny doubles of
   device memory per simulation, allocated at the first Gaussian setting).
   The beam should lie well inside the transverse boundaries.  Type 0 is
   the plane wave (default).  Kept when the seed itself changes; acts from
   the next step.  EINVAL as for the optical undulator's beam; ENOMEM if
   the corrections cannot be allocated. */
mithra_status mithra_set_seed_beam(mithra_sim *sim, const mithra_beam *beam);

/* Enqueue nsteps steps on the simulation's stream (asynchronous).  ESTATE if
   no particles were loaded (np = 0 is a valid load). */
mithra_status mithra_run(mithra_sim *sim, int64_t nsteps);

/* Wait for the stream; ENUMERIC if a non-finite momentum or diagnostic was
   produced since the last sync (the particle is then counted as lost). */
mithra_status mithra_sync(mithra_sim *sim);

/* Copy a mesh quantity to host (n[0]*n[1]*n[2] doubles, layout above). */
mithra_status mithra_get_field(mithra_sim *sim, mithra_field which, double *host);

/* For callers that cannot allocate (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): mithra_get_field without
   any device or host allocation.  The output is the same as
   mithra_get_field's, bit for bit.  E and B are computed, and float fields
   widened to double, in the library's static scratch of 6 x 2^18 doubles
   (12 MiB per GPU, held until the process ends), a chunk of whole z-planes
   at a time; a mesh whose z-plane has more than 2^18 = 262144 points
   (n[0] * n[1]) is EINVAL.  Every call on one GPU shares that GPU's scratch:
   calls that overlap on one GPU (from several threads, or simulations on
   other streams) race and must be serialized by the caller. */
mithra_status mithra_get_field_noalloc(mithra_sim *sim, mithra_field which, double *host);

/* Overwrite a stored mesh quantity (potentials at the newest or previous
   level, J, rho, rho_prev) from host doubles; E/B are derived and EINVAL. */
mithra_status mithra_set_field(mithra_sim *sim, mithra_field which, const double *host);

/* Copy the particles back in input order: pos [np][3], u [np][3] (SI), alive
   [np] (1 live, 0 lost; may be NULL); np_alive may be NULL. */
mithra_status mithra_get_particles(mithra_sim *sim, double *pos, double *u, uint8_t *alive,
                                   int64_t *np_alive);

/* The binning of the particles by cell that the deposit of the next step
   reads (the paper's deposition, section "Current Deposition", sums over the
   particles of each cell's neighbourhood; the library keeps them sorted by
   cell for that).  Cells are grouped in tiles of 8x8x8: with
   nt[a] = ceil(n[a] / 8), the key of cell (i, j, k) is
   ((k/8 * nt[1] + j/8) * nt[0] + i/8) * 512 + ((k%8) * 8 + j%8) * 8 + i%8,
   and key nkeys = nt[0] nt[1] nt[2] 512 holds the lost particles.
   keys [np]: the key of the particle in each slot of the particle buffer;
   ids [np]: its input index; starts [nkeys + 2]: the first slot of each key
   (starts[nkeys + 1] = np), so the particles of key g sit in slots
   starts[g] .. starts[g+1]-1, in no fixed order inside a key.  Any pointer
   may be NULL; *nkeys receives nkeys.  ESTATE before the first run. */
mithra_status mithra_get_bins(mithra_sim *sim, int32_t *keys, int32_t *ids, int32_t *starts,
                              int64_t *nkeys);

/* Copy the unread diagnostic rows (oldest first, at most cap) and mark them
   read; at most the last `capacity` rows are kept. */
mithra_status mithra_get_diag(mithra_sim *sim, mithra_diag_row *rows, int64_t cap,
                              int64_t *nrows);

mithra_status mithra_get_info(mithra_sim *sim, mithra_info *info);

/* Checkpoint: the potentials at the two levels the next step reads, J, rho
   (both buffers), particles, step, lost count and the running DFT of the
   power plane.  blob NULL: *bytes receives
   the size.  EINVAL if *bytes is too small or the blob belongs to another
   mesh or precision, and for a corrupt blob (negative step or particle
   count, a live particle outside the cells [2, n-3], an offset outside
   [0, 1], non-finite momenta); a refused blob changes nothing.  Blobs of
   the earlier layout without the plane spectrum are still accepted (the
   spectrum then starts from zero). */
mithra_status mithra_get_state(mithra_sim *sim, void *blob, size_t *bytes);
mithra_status mithra_set_state(mithra_sim *sim, const void *blob, size_t bytes);

/* Per-kernel timing with HIP events on the simulation's stream.  While on,
   runs launch kernel by kernel (no graph replay).  ms[k], calls[k] for
   k = 0 stencil, 1 boundary, 2 gather+push, 3 deposit, 4 scan, 5 scatter,
   6 diagnostics; totals since the last reset (reset = 1 clears them). */
mithra_status mithra_set_timing(mithra_sim *sim, int32_t on);
mithra_status mithra_get_timing(mithra_sim *sim, double *ms, int64_t *calls, int32_t nkinds,
                                int32_t reset);

/* Autotuner: times trial_steps launches of the potential-update kernel for
   each candidate tile shape (x and y columns per block, z planes per block),
   then of the push followed by the deposit for each candidate brick shape
   (tiles per brick dealt to one XCD), and keeps the fastest of each.  The
   simulation state is unchanged (the particle kernels' outputs are restored
   after every trial), and later steps give the same results bit for bit
   whatever shapes were chosen. */
mithra_status mithra_tune(mithra_sim *sim, int32_t trial_steps);

/* Sets the shapes the autotuner chooses, without timing anything: for runs
   that reuse what an earlier mithra_tune found (mithra_get_info reports it),
   and for profilers, under which trial timings mean little.  stencil_tile:
   x and y columns per block, one of 64x4, 32x8, 128x2, 64x2, 32x4, 16x16,
   256x1, 128x1, 128x4, 256x2, 64x8, and z planes per block (>= 1);
   particle_brick: tiles per brick along x, y, z (each >= 1, clipped to the
   largest tile grid).  Results do not depend on the shapes.  Returns
   MITHRA_EINVAL (and changes nothing) for a NULL array or a shape outside
   these sets. */
mithra_status mithra_set_shapes(mithra_sim *sim, const int32_t stencil_tile[3],
                                const int32_t particle_brick[3]);

const char *mithra_last_error(void);
void mithra_destroy(mithra_sim *sim);

/* ---- batch of independent simulations (parameter scans) ------------------
   nsim simulations of different meshes, bunches and undulators advance in
   lockstep: each step is one launch per kernel kind covering every
   simulation, replayed from a captured hipGraph.  Indices are 0..nsim-1. */
mithra_status mithra_batch_create(int32_t nsim, const mithra_mesh *meshes,
                                  const mithra_undulator *unds, mithra_precision prec,
                                  void *stream, mithra_batch **out);
mithra_status mithra_batch_set_particles(mithra_batch *b, int32_t sim, int64_t np,
                                         const double *pos, const double *u, double q_macro,
                                         double m_macro);
mithra_status mithra_batch_config_diag(mithra_batch *b, int32_t sim, const mithra_diag_cfg *cfg);
mithra_status mithra_batch_set_spectrum(mithra_batch *b, int32_t sim, const double *nu,
                                        int32_t nfreq);
mithra_status mithra_batch_get_spectrum(mithra_batch *b, int32_t sim, int64_t first_step,
                                        int64_t count, double *rest, double *lab);
mithra_status mithra_batch_set_seed(mithra_batch *b, int32_t sim, const mithra_seed *seed);
mithra_status mithra_batch_set_optical_undulator(mithra_batch *b, int32_t sim,
                                                 const mithra_seed *wave);
mithra_status mithra_batch_set_optical_beam(mithra_batch *b, int32_t sim, const mithra_beam *beam);
mithra_status mithra_batch_set_seed_beam(mithra_batch *b, int32_t sim, const mithra_beam *beam);
/* Autotuner of the batch (see mithra_tune): one tile shape for all
   simulations, chosen by timing the whole batched launch. */
mithra_status mithra_batch_tune(mithra_batch *b, int32_t trial_steps);
/* mithra_set_shapes for the batch: one stencil tile and one brick for all
   simulations. */
mithra_status mithra_batch_set_shapes(mithra_batch *b, const int32_t stencil_tile[3],
                                      const int32_t particle_brick[3]);
mithra_status mithra_batch_run(mithra_batch *b, int64_t nsteps);
mithra_status mithra_batch_sync(mithra_batch *b);
mithra_status mithra_batch_get_diag(mithra_batch *b, int32_t sim, mithra_diag_row *rows,
                                    int64_t cap, int64_t *nrows);
mithra_status mithra_batch_get_field(mithra_batch *b, int32_t sim, mithra_field which,
                                     double *host);
mithra_status mithra_batch_get_particles(mithra_batch *b, int32_t sim, double *pos, double *u,
                                         uint8_t *alive, int64_t *np_alive);
mithra_status mithra_batch_get_info(mithra_batch *b, int32_t sim, mithra_info *info);
mithra_status mithra_batch_set_timing(mithra_batch *b, int32_t on);
mithra_status mithra_batch_get_timing(mithra_batch *b, double *ms, int64_t *calls, int32_t nkinds,
                                      int32_t reset);
void mithra_batch_destroy(mithra_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* MITHRA_H */

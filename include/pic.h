/*
 * pic.h -- C ABI of libpic.so, the MI355X (gfx950) particle-in-cell step for
 * condensed-matter quantum plasmas of "Particle-In-Cell Simulations of Quantum
 * Plasmas" (Ngirmang, Do, Liu, Bosman, Wu; arXiv 2501.07465).
 *
 * One step of the method (Appendix A.1 cycle, Sec. 4.1 field solver):
 *   gather E_n, B_n at x_n from the Yee grid; push free (eq:borisscheme),
 *   bound (eq:modborisscheme2) and Dirac (Sec. 5) particles to v_{n+1/2},
 *   x_{n+1}; reflect at material boundaries (Sec. 3); deposit the current
 *   J^{n+1/2} (charge conserving); advance B by half a step, E by a step
 *   (eq:consteps with a unit or per-cell diagonal dielectric tensor), B by half
 *   a step.
 *
 * Conventions for every call:
 *   - Return value: PIC_OK (0) or a negative PIC_E* code; the text of the last
 *     error of a simulation is returned by pic_last_error().  No call throws,
 *     exits or prints.
 *   - Host pointers are read or written during the call only; the caller keeps
 *     ownership.  Device memory is never allocated or freed by the library: the
 *     caller passes one device arena to pic_bind() (size from pic_footprint())
 *     and keeps it alive until pic_destroy().
 *   - Work is enqueued on the HIP stream given to pic_bind(); pic_step() only
 *     enqueues.  pic_diag() and pic_sync() synchronise that stream.
 *   - SI units: metres, seconds, kilograms, coulombs, V/m, tesla.  Geometry
 *     (region centres, radii, boxes, source positions) is in cell units.
 *   - One thread at a time per simulation handle.
 */
#ifndef PIC_H
#define PIC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_MAX_SPECIES 4

/* error codes */
#define PIC_OK 0
#define PIC_EINVAL (-1)      /* invalid argument or descriptor                    */
#define PIC_ECFL (-2)        /* dt not below the stability limit eq:dtlimit        */
#define PIC_ENOMEM (-3)      /* arena smaller than pic_footprint(); host allocation */
#define PIC_ESTATE (-4)      /* call out of order (e.g. step before bind)          */
#define PIC_EDEVICE (-5)     /* HIP runtime error (text in pic_last_error)         */
#define PIC_ENONFINITE (-6)  /* a non-finite value was found (diagnostics)         */
#define PIC_ETRUNC (-7)      /* output buffer too small; *n_out holds the size     */

/* enums */
enum { PIC_FP32 = 0, PIC_FP64 = 1 };
enum { PIC_PERIODIC = 0, PIC_OPEN = 1 };
enum { PIC_FREE = 0, PIC_BOUND = 1, PIC_DIRAC = 2 };
enum { PIC_REGION_ALL = 0, PIC_REGION_BALL = 1, PIC_REGION_BOX = 2 };
enum { PIC_MOM_COLD = 0, PIC_MOM_FD = 1 };
enum { PIC_LOAD_RANDOM = 0, PIC_LOAD_QUIET = 1 };
enum { PIC_SRC_NONE = 0, PIC_SRC_SHEET = 1, PIC_SRC_POINT = 2 };

/* Grid and time stepping.  Inactive axes (index >= dims) must have n = 1. */
typedef struct {
    int dims;           /* 1, 2 or 3 active axes (x, then y, then z)                    */
    int n[3];           /* cells per axis; 1D <= 2^30, 2D <= 65535, 3D <= 2047x2047x1023 */
    double dx[3];       /* cell size per axis [m]                                        */
    double dt;          /* time step [s]; must be below eq:dtlimit                       */
    int bc[3];          /* PIC_PERIODIC or PIC_OPEN (first-order Mur) per axis           */
    int precision;      /* PIC_FP32 or PIC_FP64 for positions, fields, push and deposit  */
    int tile[3];        /* particle tile shape, powers of two (inactive axes 1)          */
    int block;          /* threads per particle-kernel workgroup: 64, 128, 256 or 512    */
    int unit;           /* most particles one particle-kernel workgroup takes from a tile */
                        /* (a tile's particles are split into units of at most this many; */
                        /* 0: one unit per tile; otherwise >= 64)                         */
    int sort_every;     /* cell sort every this many steps (>= 1)                        */
    int series_cap;     /* steps of the current time series kept on the device           */
    int track_continuity; /* 1: measure the continuity residual on every step (slower)   */
    /* soft current source J(t) = j0 sin^2(pi t/tau) sin(omega t) for 0 <= t <= tau */
    int src_kind;       /* PIC_SRC_NONE, PIC_SRC_SHEET (plane at src_index[src_axis]),   */
                        /* PIC_SRC_POINT (node src_index)                                */
    int src_comp;       /* J component 0, 1, 2                                           */
    int src_axis;       /* sheet normal                                                  */
    int src_index[3];
    double src_j0;      /* [A/m^2] */
    double src_omega;   /* [rad/s] */
    double src_tau;     /* [s]     */
    int eps_cells;      /* 1: a per-cell diagonal inverse permittivity (eq:consteps) scales  */
                        /* the E update; set by pic_load_eps_inv, unit until then.           */
                        /* 2: as 1, plus off-diagonal entries (pic_load_eps_offdiag; zero    */
                        /* until then); not with track_continuity.                           */
                        /* 0: the unit tensor (no arena space, no extra reads)               */
    int ext_field;      /* 1: a static external field (pic_load_ext_field; zero until then)   */
                        /* is added to E where the particles gather it                        */
} pic_grid_desc;

/* A species.  Free carriers follow eq:tradlorentz, bound ones eq:modlorentz
 * (diagonal omega_b^2, gamma_b), Dirac carriers the renormalised push of
 * Sec. 5.  Particles are created either by the loader (count = 0: ppc per
 * region cell, Fermi-Dirac momenta of eq:fddist, Sec. 2) or by
 * pic_load_particles (count > 0). */
typedef struct {
    int kind;            /* PIC_FREE, PIC_BOUND, PIC_DIRAC                               */
    double q;            /* charge [C]                                                   */
    double m;            /* mass [kg]; Dirac: 0 derives m_d = p_F/(2 v_F), p_F = E_F/v_F */
    double density;      /* [1/m^3]; 0 derives it from E_F (free: hbar^2(3 pi^2 n)^{2/3}/(2m); */
                         /* Dirac: E_F^2/(pi hbar^2 v_F^2) over one cell along the normal) */
    double weight;       /* real particles per macroparticle when count > 0              */
    int ppc;             /* loader: macroparticles per region cell                       */
    long long count;     /* > 0: explicit particle count (filled by pic_load_particles)  */
    int momentum;        /* PIC_MOM_COLD or PIC_MOM_FD                                   */
    double e_fermi;      /* [J] chemical potential mu = E_F of eq:fddist                 */
    double temperature;  /* [K]                                                          */
    int loading;         /* PIC_LOAD_RANDOM, or PIC_LOAD_QUIET (1D evenly spaced)        */
    double pert_amp;     /* quiet start: Lagrangian displacement amplitude (relative)     */
    int pert_mode;       /* quiet start: mode number along x                             */
    double omega0[3];    /* bound: resonance frequency per axis [rad/s]                  */
    double gamma[3];     /* bound: damping per axis [1/s]                                */
    double b_weight;     /* bound: 0 = magnetic force off, 1 = gyrotropic push           */
    double xi_radius;    /* bound: initial displacement uniform in a ball [m]            */
    double v_f;          /* Dirac: Fermi speed [m/s]                                     */
    int sheet_normal;    /* Dirac: axis normal to the sheet (velocity component removed) */
    int reflect;         /* at the region boundary (Sec. 3): 0 none, 1 specular, 2 diffusive: */
                         /* the position mirrored, the speed kept and the direction drawn     */
                         /* from the cosine law about the inward normal (free species; Dirac  */
                         /* sheets in the sheet plane, sin(theta) = 2u - 1; Philox4x32-10     */
                         /* counter (index, step, species id, 2^31), key seed)                */
    int region;          /* PIC_REGION_ALL, _BALL (rc, rr), _BOX (rlo, rhi); cell units  */
    double rc[3], rr;
    double rlo[3], rhi[3];
    int mass_per_particle; /* Dirac, Sec. 5: 1 = transverse mass m_d = p / v_F per carrier,    */
                         /* p = e / v_F with e drawn from the Fermi-Dirac distribution over the */
                         /* 2D density of states at (e_fermi, temperature); 0 = the species m   */
} pic_species_desc;

typedef struct pic_sim pic_sim;

/* Create a simulation from a grid descriptor.  Host only; validates the grid.
 * Errors: PIC_EINVAL. */
int pic_create(const pic_grid_desc* g, pic_sim** out);

/* Declare a species (Module I loader of Sec. 2 when count == 0).  Computes the
 * particle count from the region on the host; the Fermi-Dirac sampling
 * (eq:fddist by inverse CDF, counter-based Philox4x32-10 random numbers keyed by
 * seed, species id and particle index) runs on the device at pic_bind().
 * Must precede pic_bind().  Re-checks dt against eq:dtlimit with the species'
 * plasma and resonance frequencies.  Errors: PIC_EINVAL, PIC_ECFL, PIC_ESTATE. */
int pic_init_species(pic_sim* s, const pic_species_desc* d, uint64_t seed, int* species_id);

/* Device bytes the simulation needs (fields, particles, sort scratch, tile
 * current slots, tables, diagnostics).  Valid after the last species is declared. */
int pic_footprint(const pic_sim* s, size_t* bytes);

/* Bind the caller's device arena (at least pic_footprint() bytes, 256-byte
 * aligned) and HIP stream (hipStream_t, may be NULL for the default stream).
 * Zeroes the fields, uploads the loader tables and enqueues the loaders.
 * Errors: PIC_ENOMEM (arena too small), PIC_EINVAL, PIC_ESTATE, PIC_EDEVICE. */
int pic_bind(pic_sim* s, void* dev_arena, size_t bytes, void* hip_stream);

/* Copy a species' state in from host FP64 arrays: positions x[n][3] [m],
 * velocities v[n][3] (v_{n-1/2}) [m/s], and for bound species the anchor in x
 * and the displacement xi[n][3] [m]; for Dirac species with mass_per_particle
 * xi[i][0] is carrier i's transverse mass m_d [kg] (> 0); NULL otherwise.  n must equal the
 * species count.  Positions are converted to (int32 cell, in-cell offset) on
 * the host.  Synchronous.  Errors: PIC_EINVAL, PIC_ESTATE, PIC_EDEVICE. */
int pic_load_particles(pic_sim* s, int sid, const double* x, const double* v,
                       const double* xi, size_t n);

/* Copy fields in: e[3][L] and b[3][L] FP64 (B at integer time), where L is the
 * array extent of pic_field_shape().  Either may be NULL.  Synchronous.
 * Errors: PIC_EINVAL (a non-finite value; nothing is copied), PIC_ESTATE,
 * PIC_EDEVICE. */
int pic_load_fields(pic_sim* s, const double* e, const double* b);

/* Sec. 4, eq:consteps: set the spatially varying dielectric tensor, diagonal,
 * as its inverse einv[3][L] (FP64, L the extent of pic_field_shape): entry
 * [c][k][j][i] scales the curl and current terms of the update of E_c at that
 * node, E_c += dt einv (c^2 (curl B)_c - J_c / eps0).  The field energy uses
 * eps0 E^2 / (2 einv) and the Gauss residual div(E / einv).  Open faces keep
 * the vacuum Mur update (their entries are not used), so media should end
 * before them.  Needs eps_cells = 1 or 2; until this call the tensor is the
 * unit one.  Entries must be finite and positive, and dt must stay below the
 * stability limit with the fastest light speed c sqrt(max einv).
 * Synchronous.  Errors: PIC_EINVAL (eps_cells = 0, null or bad entries),
 * PIC_ECFL, PIC_ESTATE (not bound, or in a batch), PIC_EDEVICE. */
int pic_load_eps_inv(pic_sim* s, const double* einv);

/* Sec. 4, eq:consteps with a full (anisotropic, spatially varying) tensor:
 * set its off-diagonal entries e[6][L] (FP64, L the extent of
 * pic_field_shape): row a, column b != a at the E_a node, in the order
 * (a, b) = 01 02 10 12 20 21.  The E_a update gains dt sum_b e_ab U_b, where
 * U_b = c^2 (curl B)_b - J_b / eps0 is averaged onto the E_a node from the
 * E_b nodes nearest to it: the four (two where only one of a, b is an active
 * axis, one where neither is) at index offsets +s along a and -t along b,
 * s, t in {0, 1}.  On the device the term is folded into the current that
 * the field kernel reads.  Entries must be finite, and nonzero only at node
 * indices in [2, n - 2] along every open axis.  dt must stay below the
 * stability limit with c^2 scaled by the largest diagonal entry plus the
 * largest row sum of |off-diagonal entries| (a Gershgorin bound).  The
 * field energy and the Gauss residual keep using the diagonal.  Needs
 * eps_cells = 2.  Synchronous.  Errors: PIC_EINVAL (eps_cells != 2, null or
 * bad entries), PIC_ECFL, PIC_ESTATE (not bound, or in a batch), PIC_EDEVICE. */
int pic_load_eps_offdiag(pic_sim* s, const double* e);

/* Sec. 3: set the static external electrostatic field (the work-function
 * barrier) e[3][L] (FP64 V/m, L the extent of pic_field_shape), entry
 * [c][k][j][i] at the E_c node.  The particles feel E + e (the sum is formed
 * on the E nodes before the gather); the Maxwell update, the field energy and
 * the Gauss residual do not see it.  Needs ext_field = 1; zero until this
 * call.  Synchronous.  Errors: PIC_EINVAL (ext_field = 0, null or non-finite
 * entries), PIC_ESTATE (not bound, or in a batch), PIC_EDEVICE. */
int pic_load_ext_field(pic_sim* s, const double* e);

/* Array extent per axis of every field component: n for periodic (and
 * inactive) axes, n + 1 for open axes.  Component c of E sits at a half-integer
 * position along axis c; B_c at half-integer positions along the other two. */
int pic_field_shape(const pic_sim* s, int L[3]);

/* Fixed ion background for the diagnostics and, in 1D periodic runs, the
 * initial E_x from the discrete Gauss law.  mode 0: rho_ion = -rho_e(t) node
 * by node; 1: uniform -mean(rho_e); 2: uniform and E_x from Gauss (1D periodic
 * only).  Enqueued.  Errors: PIC_EINVAL, PIC_ESTATE. */
int pic_init_fields(pic_sim* s, int mode);

/* Enqueue nsteps steps of the PIC cycle of Appendix A.1 with the field solver
 * of Sec. 4.1: per step, gather E_n, B_n at x_n; push free particles by
 * eq:borisscheme (rotation eq:borisrotsol), bound ones by eq:modborisscheme2
 * (eq:modborisrotsol, or the gyrotropic rotation of eq:modborisBrot when
 * b_weight != 0) and Dirac carriers by the renormalised push of Sec. 5, to
 * v_{n+1/2} and x_{n+1} (eq:discrvel); reflect at the region boundary (Sec. 3);
 * deposit J^{n+1/2} charge-conservingly; advance B half a step, E a step
 * (eq:consteps) and B half a step, first-order Mur on open faces.  Every
 * sort_every steps (and after a load) the particles of each species are
 * cell-sorted by a stable integer radix sort.  A particle whose pushed velocity
 * is not finite is held at rest and raises the flag of PIC_DIAG_NONFINITE_FLAG.
 * Returns enqueue errors only; device-side errors surface at the next
 * pic_diag/pic_sync.  Errors: PIC_ESTATE, PIC_EDEVICE. */
int pic_step(pic_sim* s, int nsteps);

/* Capture the steps in HIP graphs (one graph per sort period) and replay them
 * in pic_step.  on = 0 returns to plain launches. */
int pic_use_graphs(pic_sim* s, int on);

/* Diagnostics of the state (FP64, computed on the device).  Synchronises the
 * stream.  The energies are those of the fields (with the dielectric of
 * eq:consteps weighting the electric part) and of the macroparticles
 * (m w |v|^2 / 2, the carrier energy of eq:fddist); the Gauss residual checks
 * the law the field solver of Sec. 4.1 keeps from its initial state.
 *   PIC_DIAG_FIELD_ENERGY       1 value  [J (per m^(3-dims))]
 *   PIC_DIAG_KINETIC_ENERGY     1 value per species (arg = species id, -1 all)
 *   PIC_DIAG_GAUSS_RESIDUAL     2 values: max|div E - rho/eps0|, max|rho_e|/eps0
 *   PIC_DIAG_CONTINUITY         2 values: last step's max|drho/dt + div J|, max|rho|/dt
 *   PIC_DIAG_CURRENT_SERIES     3 per recorded step: sum q w v_{n+1/2}
 *   PIC_DIAG_PARTICLE_COUNT     1 value per species
 *   PIC_DIAG_STEP               1 value: steps done
 *   PIC_DIAG_OVERFLOW           1 value: particles that left their tile window
 *   PIC_DIAG_EXPORT_PARTICLES   species arg: x[n][3], v[n][3], xi[n][3] (9n values; Dirac
 *                               species with mass_per_particle: m_d in xi[i][0])
 *   PIC_DIAG_EXPORT_FIELDS      e[3][L], b[3][L]
 *   PIC_DIAG_EXPORT_CURRENT     the last step's particle current J[3][L] (needs track_continuity)
 *   PIC_DIAG_KEYS               species arg: the cell key of each particle (as doubles)
 *   PIC_DIAG_NONFINITE_FLAG     1 value: 1 if some step since pic_bind pushed a particle to a
 *                               non-finite velocity (that particle was held at rest), else 0
 * Errors: PIC_ETRUNC (with *n_out set), PIC_EINVAL, PIC_ESTATE, PIC_EDEVICE,
 * PIC_ENONFINITE (a non-finite field energy or kinetic energy). */
enum {
    PIC_DIAG_FIELD_ENERGY = 0,
    PIC_DIAG_KINETIC_ENERGY = 1,
    PIC_DIAG_GAUSS_RESIDUAL = 2,
    PIC_DIAG_CONTINUITY = 3,
    PIC_DIAG_CURRENT_SERIES = 4,
    PIC_DIAG_PARTICLE_COUNT = 5,
    PIC_DIAG_STEP = 6,
    PIC_DIAG_OVERFLOW = 7,
    PIC_DIAG_EXPORT_PARTICLES = 8,
    PIC_DIAG_EXPORT_FIELDS = 9,
    PIC_DIAG_EXPORT_CURRENT = 10,
    PIC_DIAG_KEYS = 11,
    PIC_DIAG_NONFINITE_FLAG = 12
};
int pic_diag(pic_sim* s, int kind, int arg, double* out, size_t cap, size_t* n_out);

/* Sec. 2 relaxation study: histogram of the macroparticle kinetic energies
 * m |v|^2 / 2 (FP64 from the stored velocities) of species sid, counts[b] for
 * b < nbins the energies in [b, b + 1) * e_max / nbins joules, counts[nbins]
 * those at or above e_max (nbins + 1 entries, host memory).  Macroparticles
 * are counted, not weighted.  Synchronises.  Errors: PIC_EINVAL (species id,
 * nbins outside 1 .. 4096, e_max not positive, null counts), PIC_ESTATE,
 * PIC_EDEVICE. */
int pic_energy_histogram(pic_sim* s, int sid, double e_max, int nbins, uint64_t* counts);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid it): pic_energy_histogram with its
 * device counters in a static array of the library (4097 counts of 64 bits, one
 * copy per GPU, held until the process ends) instead of the simulation's arena.
 * Same arguments, results and errors as pic_energy_histogram; nbins beyond 4096
 * is refused with PIC_EINVAL.  The call allocates nothing and clears the counters
 * it uses; all calls on one GPU share them, so calls that overlap on one GPU
 * (several host threads, several streams) race.  Synchronises the simulation's
 * stream.  Errors: PIC_EINVAL, PIC_ESTATE, PIC_EDEVICE. */
int pic_energy_histogram_static(pic_sim* s, int sid, double e_max, int nbins, uint64_t* counts);

/* Run nsteps plain (non-graph) steps with HIP events recorded on the bound
 * stream around each launch and return average device times in milliseconds:
 * out[0] particle kernel, out[1] field kernel, out[2] one cell sort of all
 * species (0 if none ran), out[3] number of sorts timed.  Synchronises.
 * Errors: PIC_ESTATE, PIC_EDEVICE. */
int pic_time_kernels(pic_sim* s, int nsteps, double out[4]);

/* Wait for all enqueued work.  Errors: PIC_EDEVICE. */
int pic_sync(pic_sim* s);

/* Move the simulation's later work to another HIP stream (on the same device):
 * the new stream first waits for everything enqueued on the old one so far
 * (an event; the host does not wait).  Not while the simulation is in a batch.
 * Errors: PIC_EINVAL, PIC_ESTATE, PIC_EDEVICE. */
int pic_set_stream(pic_sim* s, void* hip_stream);

/* Number of particles of a species (host value). */
long long pic_species_count(const pic_sim* s, int sid);

/* Text of the last error on this simulation ("" if none).  s may be NULL for
 * errors of pic_create. */
const char* pic_last_error(const pic_sim* s);

/* Release host resources.  Null-safe; does not touch the caller's arena. */
void pic_destroy(pic_sim* s);

/* ---- Batched form: many independent simulations advanced by the same
 * persistent kernels (one launch per phase for the whole batch).  The batch has
 * max_sims fixed slots; one HIP graph per sort period holds the particle and
 * field launches over every slot (an empty slot is passed over), and each
 * member's sorts are a graph of its own, captured when it joins.  Joining and
 * leaving write the member's table entry on the batch stream (the host does not
 * wait); the step graph is captured again only when a joining member needs
 * more than it was captured for (larger LDS windows or block, a kernel
 * variant, or a full-tensor permittivity).  All members share dims, precision
 * and sort period. ---- */
typedef struct pic_batch pic_batch;

/* Device bytes of the batch tables for up to max_sims members. */
int pic_batch_footprint(int max_sims, int dims, size_t* bytes);
/* Create a batch over a caller-owned device arena and a non-null stream. */
int pic_batch_create(int max_sims, int dims, int precision, void* dev_arena, size_t bytes,
                     void* hip_stream, pic_batch** out);
/* Add or remove a bound simulation (bound to the batch stream).  A member must
 * be at a multiple of its sort period when added.  A removed simulation can be
 * stepped, read or moved to another stream (pic_set_stream) on its own; its
 * diagnostics wait only for its own work when it is moved first.  Errors:
 * PIC_EINVAL, PIC_ESTATE, PIC_ENOMEM, PIC_EDEVICE. */
int pic_batch_add(pic_batch* b, pic_sim* s);
int pic_batch_remove(pic_batch* b, pic_sim* s);
/* Advance every member by k steps (k a multiple of the members' common sort
 * period); only enqueues. */
int pic_batch_step(pic_batch* b, int k);
int pic_batch_size(const pic_batch* b);
/* How many times the step graph has been captured (membership changes that
 * the captured graph covers do not capture it again). */
int pic_batch_captures(const pic_batch* b);
const char* pic_batch_last_error(const pic_batch* b);
void pic_batch_destroy(pic_batch* b);

#ifdef __cplusplus
}
#endif
#endif

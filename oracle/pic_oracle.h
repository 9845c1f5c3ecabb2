/*
 * pic_oracle.h -- plain FP64 CPU oracle for the particle-in-cell step of
 * "Particle-In-Cell Simulations of Quantum Plasmas" (Ngirmang, Do, Liu, Bosman, Wu;
 * arXiv 2501.07465).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP library; the product path never
 * links it.
 *
 * Units are SI throughout the interface: positions in metres, velocities in
 * m/s, fields in V/m and T, charge in C, mass in kg.  Internally positions are
 * kept in cell units (x / dx).
 *
 * Every function names the passage of the paper it follows.  Where the paper is
 * silent or its printed formula is garbled the reading taken is stated at the
 * function.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_FREE = 0, OR_BOUND = 1, OR_DIRAC = 2 };
enum { OR_REGION_ALL = 0, OR_REGION_BALL = 1, OR_REGION_BOX = 2 };
enum { OR_SRC_NONE = 0, OR_SRC_SHEET = 1, OR_SRC_POINT = 2 };
enum { OR_MOM_COLD = 0, OR_MOM_FD = 1 };
enum { OR_LOAD_RANDOM = 0, OR_LOAD_QUIET = 1 };

typedef struct {
    int dims;            /* 1, 2 or 3 active axes (x, then y, then z)          */
    int n[3];            /* cells per axis; inactive axes must be 1           */
    double dx[3];        /* cell size per axis [m]                            */
    double dt;           /* time step [s]                                     */
    int periodic[3];     /* 1: periodic, 0: open (first-order Mur)            */
    int tile[3];         /* tile shape used by the cell key                    */
    int sort_every;      /* stable cell sort every this many steps (>=1)      */
    /* soft current source J_src(t) = j0 sin^2(pi t / tau) sin(omega t), 0<=t<=tau */
    int src_kind;        /* OR_SRC_*                                          */
    int src_comp;        /* 0,1,2: which J component                          */
    int src_axis;        /* sheet: normal axis                                */
    int src_index[3];    /* sheet: src_index[src_axis]; point: (i,j,k)        */
    double src_j0;       /* [A/m^2]                                           */
    double src_omega;    /* [rad/s]                                           */
    double src_tau;      /* [s]                                               */
} or_grid;

typedef struct {
    int kind;            /* OR_FREE, OR_BOUND, OR_DIRAC                       */
    double q;            /* charge [C]                                        */
    double m;            /* mass [kg]; Dirac: transverse mass m_d             */
    double weight;       /* real particles per macroparticle (per m^(3-dims)) */
    double omega0_sq[3]; /* bound: diagonal omega_b^2 [1/s^2]                 */
    double gamma[3];     /* bound: diagonal gamma_b [1/s]                     */
    double b_weight;     /* bound: 0 (magnetic force off) or 1 (gyrotropic)   */
    double v_f;          /* Dirac: Fermi speed [m/s]                          */
    int sheet_normal;    /* Dirac: axis whose velocity component is removed, or -1 */
    int reflect;         /* 0: none; 1: specular, 2: diffusive (Lambert) scattering */
                         /* at the region boundary (Sec. 3)                   */
    int region;          /* OR_REGION_*                                       */
    double rc[3], rr;    /* ball centre and radius [cells]                    */
    double rlo[3], rhi[3]; /* box corners [cells]                             */
    uint64_t seed;       /* Philox key of the diffusive draws                 */
    int mass_per_particle; /* Dirac: 1 = transverse mass m_d = p / v_F per particle */
                         /* (carried in xi[i][0]); 0 = the species mass m     */
} or_species;

typedef struct {
    int ppc;             /* macroparticles per cell of the region            */
    int momentum;        /* OR_MOM_COLD or OR_MOM_FD                          */
    double e_fermi;      /* [J]                                               */
    double temperature;  /* [K]                                               */
    double density;      /* [1/m^3]; 0 -> derived from e_fermi                */
    int loading;         /* OR_LOAD_RANDOM or OR_LOAD_QUIET (1D only)         */
    double pert_amp;     /* quiet start: Lagrangian displacement amplitude    */
    int pert_mode;       /* quiet start: mode number along x                  */
    double xi_radius;    /* bound: initial displacement ball radius [m]       */
    uint64_t seed;
} or_init;

typedef struct or_sim or_sim;

/* ---- constants and closed forms ------------------------------------------------ */
double or_const(int which); /* 0 qe, 1 me, 2 c, 3 eps0, 4 hbar, 5 kB, 6 mu0 */
double or_fermi_energy(double density, double mass);
double or_density_from_fermi(double e_fermi, double mass);
double or_dirac_mass(double e_fermi, double v_f);
double or_dirac_density2d(double e_fermi, double v_f);
double or_dt_limit(double omega_b, double omega_p, const double dx[3], int dims);

/* ---- random numbers: Philox4x32-10 and the 53-bit uniform built on it ---------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_u53(uint32_t a, uint32_t b);

/* ---- single-particle building blocks (exported for unit tests) ----------------- */
void or_boris_matrix(const double b[3], double R[9]);
void or_gyro_matrix(const double b[3], const double g[3], double R[9]);
void or_push_free(double qm, double dt, const double E[3], const double B[3], double v[3]);
void or_push_bound(double qm, double dt, const double w2[3], const double gam[3],
                   double bw, const double E[3], const double B[3],
                   const double xi[3], double v[3]);
void or_push_dirac(double qm, double dt, double v_f, int normal,
                   const double E[3], const double B[3], double v[3]);
int  or_reflect(const or_species* s, int dims, double X[3], double v[3]);
/* Diffusive scattering of a reflected particle: the speed |v| kept, the direction
 * drawn from the cosine (Lambert) law about the inward unit normal n, with the
 * two uniforms u[0], u[1] in (0,1). */
void or_lambert(const double n[3], const double u[2], double v[3]);
/* Dirac carriers: the in-sheet cosine law, sin(theta) = 2 u[0] - 1, about the
 * in-sheet inward normal n, tangent e_normal x n; the speed kept. */
void or_lambert2d(const double n[3], int normal, const double u[2], double v[3]);
/* The two uniforms of the diffusive draw of particle p of species sid in step
 * `step` (Philox4x32-10, counter (p, step, sid, 0x80000000), key seed). */
void or_scatter_uniforms(uint64_t seed, uint32_t p, uint32_t step, uint32_t sid, double u[2]);
int  or_fd_sample_speeds(double e_fermi, double kT, double mass, size_t n,
                         const double* u, double* speed);
/* Energies of Dirac carriers (2D density of states ~ e) under eq:fddist. */
int  or_dirac_sample_energies(double e_fermi, double kT, size_t n, const double* u, double* e);

/* ---- simulation -------------------------------------------------------------- */
int  or_create(const or_grid* g, or_sim** out);
void or_destroy(or_sim* s);
int  or_add_species(or_sim* s, const or_species* sp, size_t n,
                    const double* x, const double* v, const double* xi);
int  or_init_species(or_sim* s, const or_species* sp, const or_init* ini, int* sid);
size_t or_count(const or_sim* s, int sid);
double or_species_weight(const or_sim* s, int sid);
int  or_get_particles(const or_sim* s, int sid, double* x, double* v, double* xi);
int  or_keys(const or_sim* s, int sid, int32_t* keys);
size_t or_field_len(const or_sim* s);
void or_field_shape(const or_sim* s, int L[3]);
int  or_get_fields(const or_sim* s, double* e, double* b);   /* [3][L] each */
/* Sec. 4, eq:consteps with a diagonal, spatially varying dielectric tensor:
 * einv[3][L] holds the inverse permittivity of component c at the E_c node
 * (NULL restores the unit tensor).  Entries must be finite and positive. */
int  or_set_eps_inv(or_sim* s, const double* einv);
/* The off-diagonal entries of the inverse dielectric tensor, e[6][L]: row a,
 * column b != a at the E_a node, in the order 01 02 10 12 20 21 (NULL: none).
 * The update term of component b is averaged onto the E_a node from its four
 * (two, one) nearest E_b nodes.  Entries must be finite, and nonzero only at
 * node indices in [2, n - 2] on every open axis. */
int  or_set_eps_offdiag(or_sim* s, const double* e);
/* Sec. 2 relaxation study: macroparticle kinetic-energy histogram of species
 * sid, nbins bins over [0, e_max) joules plus counts[nbins] at or above it. */
int  or_energy_histogram(const or_sim* s, int sid, double e_max, int nbins, uint64_t* counts);
/* Sec. 3: a static external electrostatic field e[3][L] at the E_c nodes (the
 * work-function barrier), felt by the particles (gathered like E) and outside
 * the Maxwell update and the field diagnostics.  NULL removes it. */
int  or_set_ext_field(or_sim* s, const double* e);
int  or_set_fields(or_sim* s, const double* e, const double* b);
int  or_get_current(const or_sim* s, double* j);             /* last particle J, [3][L] */
int  or_get_rho(const or_sim* s, double* rho);               /* particle rho at nodes, [L] */
int  or_gather_at(const or_sim* s, const double x[3], double E[3], double B[3]);
int  or_set_ion_background(or_sim* s, int uniform);
int  or_gauss_init_1d(or_sim* s);
int  or_step(or_sim* s, int nsteps);
void or_track_continuity(or_sim* s, int on);
int  or_sort(or_sim* s);
long or_steps_done(const or_sim* s);

/* diagnostics (FP64) */
double or_field_energy(const or_sim* s);
double or_kinetic_energy(const or_sim* s, int sid);
double or_gauss_residual(const or_sim* s, double* scale);
int    or_current_series(const or_sim* s, double* out, size_t cap, size_t* n);
double or_last_continuity_residual(const or_sim* s, double* scale);

#ifdef __cplusplus
}
#endif
#endif

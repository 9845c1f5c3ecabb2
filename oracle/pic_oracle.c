/*
 * pic_oracle.c -- plain FP64 CPU oracle of the particle-in-cell step of
 * "Particle-In-Cell Simulations of Quantum Plasmas" (arXiv 2501.07465).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  It shares no code with the HIP library.
 * It is written for a reader checking it against the paper: one particle at a
 * time, one grid node at a time, in the order the paper states the cycle
 * (gather at x_n, push to v_{n+1/2} and x_{n+1}, deposit J, advance the
 * fields), with no blocking, fusion or reordering.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so each
 * product and sum is rounded exactly as written).
 *
 * Readings of points the paper leaves open or prints garbled are marked
 * "Reading:" at the place they are used.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Physical constants (CODATA 2018; e, c, hbar, kB exact).                    */
/* ------------------------------------------------------------------------- */
static const double QE = 1.602176634e-19;
static const double ME = 9.1093837015e-31;
static const double CLIGHT = 299792458.0;
static const double EPS0 = 8.8541878128e-12;
static const double HBAR = 1.054571817e-34;
static const double KB = 1.380649e-23;
static const double PI = 3.14159265358979323846;

double or_const(int which)
{
    switch (which) {
    case 0: return QE;
    case 1: return ME;
    case 2: return CLIGHT;
    case 3: return EPS0;
    case 4: return HBAR;
    case 5: return KB;
    case 6: return 1.0 / (EPS0 * CLIGHT * CLIGHT);
    default: return NAN;
    }
}

/* ------------------------------------------------------------------------- */
/* Closed forms                                                              */
/* ------------------------------------------------------------------------- */

/* Fermi energy of a free-electron gas of density N (Sec. 2, FD relaxation
 * study).  Reading: the printed exponent 3/2 is a typo for 2/3; with 2/3,
 * N = 5.9e28 m^-3 gives 5.53 eV, the usual value for such metals. */
double or_fermi_energy(double density, double mass)
{
    return HBAR * HBAR / (2.0 * mass) * pow(3.0 * PI * PI * density, 2.0 / 3.0);
}

/* Inverse of or_fermi_energy. */
double or_density_from_fermi(double e_fermi, double mass)
{
    return pow(2.0 * mass * e_fermi / (HBAR * HBAR), 1.5) / (3.0 * PI * PI);
}

/* Averaged transverse mass of the Dirac carriers, m_d = p_F / (2 v_F) with
 * p_F = E_F / v_F (Sec. 5, graphene disk example). */
double or_dirac_mass(double e_fermi, double v_f)
{
    return (e_fermi / v_f) / (2.0 * v_f);
}

/* Sheet density of a Dirac gas with fourfold degeneracy:
 * n_2D = k_F^2 / pi with k_F = E_F / (hbar v_F).  Reading: the paper quotes
 * densities but not this relation; it is the standard graphene result. */
double or_dirac_density2d(double e_fermi, double v_f)
{
    double kf = e_fermi / (HBAR * v_f);
    return kf * kf / PI;
}

/* Stability limit of the modified Boris scheme coupled to Yee (eq:dtlimit):
 * dt < 1 / sqrt(omega_b^2/4 + omega_p^2/4 + c^2 sum_l 1/dx_l^2), summed over
 * the active axes. */
double or_dt_limit(double omega_b, double omega_p, const double dx[3], int dims)
{
    double s = 0.0;
    for (int a = 0; a < dims; ++a) s += 1.0 / (dx[a] * dx[a]);
    return 1.0 / sqrt(0.25 * omega_b * omega_b + 0.25 * omega_p * omega_p +
                      CLIGHT * CLIGHT * s);
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its        */
/* published definition: ten rounds of two 32x32->64 multiplies with a Weyl   */
/* key schedule.                                                             */
/* ------------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform double in (0,1) from 53 random bits: 27 from a, 26 from b. */
double or_u53(uint32_t a, uint32_t b)
{
    uint64_t k = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)k + 0.5) * (1.0 / 9007199254740992.0);
}

/* Six uniforms for macroparticle p of species sid: counter (p_lo, p_hi, sid,
 * call), key = seed; two Philox calls, each giving two 53-bit uniforms. */
static void draw6(uint64_t seed, int sid, uint64_t p, double u[6])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t call = 0; call < 3; ++call) {
        uint32_t ctr[4] = {(uint32_t)p, (uint32_t)(p >> 32), (uint32_t)sid, call};
        uint32_t r[4];
        or_philox4x32_10(ctr, key, r);
        u[2 * call + 0] = or_u53(r[0], r[1]);
        u[2 * call + 1] = or_u53(r[2], r[3]);
    }
}

/* ------------------------------------------------------------------------- */
/* Fermi-Dirac speeds (eq:fddist).                                            */
/* f(v) d^3v ~ 1 / (1 + exp((m v^2/2 - mu)/kT)) d^3v with mu = E_F.           */
/* In energy the isotropic density is p(e) ~ sqrt(e) f(e).  Reading: the      */
/* paper names a custom loader but no sampling method; the oracle samples by  */
/* inverse CDF.  With x = sqrt(e / e_max), e_max = mu + 40 kT, the density is */
/* p(x) ~ x^2 f(e_max x^2), smooth at 0.  The CDF is tabulated by the          */
/* trapezoid rule on 65536 uniform x-intervals and inverted by bisection and  */
/* linear interpolation.  At T = 0 the closed form e = E_F u^(2/3) is used.    */
/* ------------------------------------------------------------------------- */
#define FD_NTAB 65536

typedef struct {
    double e_max;
    double cdf[FD_NTAB + 1];
} fd_table;

/* dos2d = 0: the 3D free-carrier density of states sqrt(e), p(x) ~ x^2 f; dos2d = 1: the 2D Dirac
 * density of states e, p(x) ~ x^3 f (de = 2 e_max x dx). */
static void fd_table_build(fd_table* t, double mu, double kT, int dos2d)
{
    t->e_max = mu + 40.0 * kT;
    double prev = 0.0; /* p(0) = 0 */
    t->cdf[0] = 0.0;
    for (int k = 1; k <= FD_NTAB; ++k) {
        double x = (double)k / (double)FD_NTAB;
        double e = t->e_max * x * x;
        double p = (dos2d ? x * x * x : x * x) / (1.0 + exp((e - mu) / kT));
        t->cdf[k] = t->cdf[k - 1] + 0.5 * (prev + p) * (1.0 / (double)FD_NTAB);
        prev = p;
    }
    double total = t->cdf[FD_NTAB];
    for (int k = 0; k <= FD_NTAB; ++k) t->cdf[k] /= total;
}

static double fd_table_energy(const fd_table* t, double u)
{
    int lo = 0, hi = FD_NTAB;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (t->cdf[mid] <= u) lo = mid; else hi = mid;
    }
    double span = t->cdf[lo + 1] - t->cdf[lo];
    double frac = span > 0.0 ? (u - t->cdf[lo]) / span : 0.0;
    double x = ((double)lo + frac) / (double)FD_NTAB;
    return t->e_max * x * x;
}

static double fd_speed(const fd_table* t, double e_fermi, double kT, double mass, double u)
{
    double e;
    if (kT > 0.0) e = fd_table_energy(t, u);
    else e = e_fermi * pow(u, 2.0 / 3.0);
    return sqrt(2.0 * e / mass);
}

/* Dirac carriers: energies under the 2D density of states, p(e) ~ e f(e)
 * (Sec. 5 with eq:fddist; reading: the paper loads Dirac carriers at v_F
 * without saying how their momenta are drawn).  At T = 0, e = E_F sqrt(u). */
static double dirac_energy(const fd_table* t, double e_fermi, double kT, double u)
{
    if (kT > 0.0) return fd_table_energy(t, u);
    return e_fermi * sqrt(u);
}

int or_dirac_sample_energies(double e_fermi, double kT, size_t n, const double* u, double* e)
{
    fd_table* t = NULL;
    if (kT > 0.0) {
        t = (fd_table*)malloc(sizeof(fd_table));
        if (!t) return -2;
        fd_table_build(t, e_fermi, kT, 1);
    }
    for (size_t i = 0; i < n; ++i) e[i] = dirac_energy(t, e_fermi, kT, u[i]);
    free(t);
    return 0;
}

int or_fd_sample_speeds(double e_fermi, double kT, double mass, size_t n,
                        const double* u, double* speed)
{
    fd_table* t = NULL;
    if (kT > 0.0) {
        t = (fd_table*)malloc(sizeof(fd_table));
        if (!t) return -1;
        fd_table_build(t, e_fermi, kT, 0);
    }
    for (size_t i = 0; i < n; ++i) speed[i] = fd_speed(t, e_fermi, kT, mass, u[i]);
    free(t);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Pushers (Appendix A).                                                      */
/* ------------------------------------------------------------------------- */

/* Rotation of the standard Boris scheme, eq:borisrotsol:
 * R = [I(1-|b|^2) + 2 b(x)b + 2 eps(b)] / (1+|b|^2), b = dt q B / (2m),
 * with eps(v) the matrix printed below eq:borisrotsol, eps(b) u = u x b. */
void or_boris_matrix(const double b[3], double R[9])
{
    double bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double eps[9] = {0.0, b[2], -b[1],
                     -b[2], 0.0, b[0],
                     b[1], -b[0], 0.0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double id = (r == c) ? 1.0 : 0.0;
            R[3 * r + c] = (id * (1.0 - bb) + 2.0 * b[r] * b[c] + 2.0 * eps[3 * r + c]) / (1.0 + bb);
        }
}

/* Solve A y = r for a 3x3 system by Gaussian elimination with partial pivoting. */
static void solve3(const double Ain[9], const double rin[3], double y[3])
{
    double A[9], r[3];
    memcpy(A, Ain, sizeof(A));
    memcpy(r, rin, sizeof(r));
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int row = col + 1; row < 3; ++row)
            if (fabs(A[3 * row + col]) > fabs(A[3 * piv + col])) piv = row;
        if (piv != col) {
            for (int c = 0; c < 3; ++c) {
                double t = A[3 * col + c]; A[3 * col + c] = A[3 * piv + c]; A[3 * piv + c] = t;
            }
            double t = r[col]; r[col] = r[piv]; r[piv] = t;
        }
        for (int row = col + 1; row < 3; ++row) {
            double f = A[3 * row + col] / A[3 * col + col];
            for (int c = col; c < 3; ++c) A[3 * row + c] -= f * A[3 * col + c];
            r[row] -= f * r[col];
        }
    }
    for (int row = 2; row >= 0; --row) {
        double s = r[row];
        for (int c = row + 1; c < 3; ++c) s -= A[3 * row + c] * y[c];
        y[row] = s / A[3 * row + row];
    }
}

/* Rotation for a bound species with the magnetic force on (Appendix A.2,
 * eq:modborisBrot).  Reading: the rotation equation is
 * (v+ - v-) = (eps(b) - G)(v+ + v-) with b = (dt/2)(q/m)B and G = (dt/2) gamma
 * (the printed q/m on gamma is a typo), i.e. L- v+ = L+ v- with
 * L- = I + G - eps(b), L+ = I - G + eps(b).  The oracle forms R = L-^{-1} L+
 * column by column with a direct 3x3 solve; the printed closed-form numerator
 * is not used (with gamma = 0 it does not reduce to eq:borisrotsol). */
void or_gyro_matrix(const double b[3], const double g[3], double R[9])
{
    double eps[9] = {0.0, b[2], -b[1],
                     -b[2], 0.0, b[0],
                     b[1], -b[0], 0.0};
    double Lm[9], Lp[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double id = (r == c) ? 1.0 : 0.0;
            double G = (r == c) ? g[r] : 0.0;
            Lm[3 * r + c] = id + G - eps[3 * r + c];
            Lp[3 * r + c] = id - G + eps[3 * r + c];
        }
    for (int c = 0; c < 3; ++c) {
        double col[3] = {Lp[c], Lp[3 + c], Lp[6 + c]}, y[3];
        solve3(Lm, col, y);
        R[c] = y[0]; R[3 + c] = y[1]; R[6 + c] = y[2];
    }
}

static void matvec(const double R[9], const double u[3], double y[3])
{
    for (int r = 0; r < 3; ++r)
        y[r] = R[3 * r + 0] * u[0] + R[3 * r + 1] * u[1] + R[3 * r + 2] * u[2];
}

/* Standard Boris scheme for a free species, eq:borisscheme with the rotation
 * eq:borisrotsol.  v holds v_{n-1/2} on entry and v_{n+1/2} on exit.  (The
 * position update x_{n+1} = x_n + dt v_{n+1/2} of eq:discrvel is done by the
 * caller; the printed "x_{n+1} = dt v" drops the x_n.) */
void or_push_free(double qm, double dt, const double E[3], const double B[3], double v[3])
{
    double vm[3], vp[3], b[3], R[9];
    for (int a = 0; a < 3; ++a) vm[a] = v[a] + 0.5 * dt * qm * E[a];
    for (int a = 0; a < 3; ++a) b[a] = 0.5 * dt * qm * B[a];
    or_boris_matrix(b, R);
    matvec(R, vm, vp);
    for (int a = 0; a < 3; ++a) v[a] = vp[a] + 0.5 * dt * qm * E[a];
}

/* Modified Boris scheme for a bound species (eq:modborisscheme2, Appendix
 * A.2).  The acceleration (q/m)E_n - omega_b^2 . x_b is applied as two half
 * kicks around the damping rotation R(gamma) of eq:modborisrotsol.
 * Readings: the first kick carries dt/2 (the printed scheme drops it; the
 * half-step definition eq:modborisvpm has it); x_b is the displacement xi of
 * the particle from its anchor; the magnetic force is weighted by b_weight
 * (0: eq:modborisrotsol, 1: gyrotropic rotation). */
void or_push_bound(double qm, double dt, const double w2[3], const double gam[3],
                   double bw, const double E[3], const double B[3],
                   const double xi[3], double v[3])
{
    double acc[3], vm[3], vp[3];
    for (int a = 0; a < 3; ++a) acc[a] = qm * E[a] - w2[a] * xi[a];
    for (int a = 0; a < 3; ++a) vm[a] = v[a] + 0.5 * dt * acc[a];
    if (bw != 0.0) {
        double b[3], g[3], R[9];
        for (int a = 0; a < 3; ++a) b[a] = 0.5 * dt * qm * bw * B[a];
        for (int a = 0; a < 3; ++a) g[a] = 0.5 * dt * gam[a];
        or_gyro_matrix(b, g, R);
        matvec(R, vm, vp);
    } else {
        for (int a = 0; a < 3; ++a)
            vp[a] = (1.0 - 0.5 * gam[a] * dt) / (1.0 + 0.5 * gam[a] * dt) * vm[a];
    }
    for (int a = 0; a < 3; ++a) v[a] = vp[a] + 0.5 * dt * acc[a];
}

/* Dirac carriers (Sec. 5): Boris push with the transverse mass, then the
 * velocity is renormalised to v_F.  Readings: the component along the sheet
 * normal is removed before renormalising (carriers stay in the sheet); if the
 * intermediate velocity vanishes the previous direction is kept. */
void or_push_dirac(double qm, double dt, double v_f, int normal,
                   const double E[3], const double B[3], double v[3])
{
    double vold[3] = {v[0], v[1], v[2]};
    double w[3] = {v[0], v[1], v[2]};
    or_push_free(qm, dt, E, B, w);
    if (normal >= 0 && normal < 3) w[normal] = 0.0;
    double mag = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (mag > 0.0) {
        for (int a = 0; a < 3; ++a) v[a] = v_f * (w[a] / mag);
    } else {
        for (int a = 0; a < 3; ++a) v[a] = vold[a];
    }
}

/* ------------------------------------------------------------------------- */
/* Material boundary (Sec. 3, conditional boundary with specular scattering). */
/* Reading: the particle is mirrored back into its region; for a ball the    */
/* mirror is radial, x' = c + (2R - r) r_hat, v' = v - 2 (v.r_hat) r_hat with */
/* r_hat at the escaped point; for a box each face is a mirror plane.  X is   */
/* in cell units; v in m/s.  Returns 1 if the particle was reflected.        */
/* ------------------------------------------------------------------------- */
int or_reflect(const or_species* s, int dims, double X[3], double v[3])
{
    int hit = 0;
    if (s->region == OR_REGION_BALL) {
        double r2 = 0.0;
        for (int a = 0; a < dims; ++a) r2 += (X[a] - s->rc[a]) * (X[a] - s->rc[a]);
        if (r2 > s->rr * s->rr) {
            double r = sqrt(r2);
            double rhat[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < dims; ++a) rhat[a] = (X[a] - s->rc[a]) / r;
            /* v is in m/s and X in cell units; with unequal dx the normal
             * differs between the two, so the oracle requires equal dx for
             * ball regions (checked at species creation). */
            double vn = 0.0;
            for (int a = 0; a < dims; ++a) vn += v[a] * rhat[a];
            for (int a = 0; a < dims; ++a) {
                X[a] = s->rc[a] + (2.0 * s->rr - r) * rhat[a];
                v[a] = v[a] - 2.0 * vn * rhat[a];
            }
            hit = 1;
        }
    } else if (s->region == OR_REGION_BOX) {
        for (int a = 0; a < dims; ++a) {
            if (X[a] > s->rhi[a]) { X[a] = 2.0 * s->rhi[a] - X[a]; v[a] = -v[a]; hit = 1; }
            else if (X[a] < s->rlo[a]) { X[a] = 2.0 * s->rlo[a] - X[a]; v[a] = -v[a]; hit = 1; }
        }
    }
    return hit;
}

/* ------------------------------------------------------------------------- */
/* Diffusive scattering at the material boundary (Sec. 3 names specular and  */
/* diffusive models; the paper gives no formula).  Reading: the collision is  */
/* elastic, the position is mirrored as in the specular case, and the new    */
/* direction follows the cosine law about the inward normal: cos(theta) =     */
/* sqrt(u0), phi = 2 pi u1, on the basis (n, t1, t2) with t1 = n x e_k / |.|, */
/* e_k the axis of the smallest |n_k| (lowest k on ties), t2 = n x t1.        */
/* ------------------------------------------------------------------------- */
void or_lambert(const double n[3], const double u[2], double v[3])
{
    double speed = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    int k = 0;
    for (int a = 1; a < 3; ++a)
        if (fabs(n[a]) < fabs(n[k])) k = a;
    double e[3] = {0.0, 0.0, 0.0};
    e[k] = 1.0;
    double t1[3] = {n[1] * e[2] - n[2] * e[1], n[2] * e[0] - n[0] * e[2], n[0] * e[1] - n[1] * e[0]};
    double l = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    for (int a = 0; a < 3; ++a) t1[a] /= l;
    double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
    double ct = sqrt(u[0]), st = sqrt(1.0 - u[0]);
    double ph = 2.0 * PI * u[1];
    double cp = cos(ph), sp = sin(ph);
    for (int a = 0; a < 3; ++a) v[a] = speed * (ct * n[a] + st * (cp * t1[a] + sp * t2[a]));
}

/* Dirac carriers move in their sheet, so their diffusive draw is two-dimensional.  Reading: the
 * in-sheet cosine law, sin(theta) = 2 u0 - 1 (uniform), about the in-sheet inward normal n
 * (n has no component along the sheet normal axis `normal`), with the tangent t = e_normal x n;
 * the speed (v_F) is kept. */
void or_lambert2d(const double n[3], int normal, const double u[2], double v[3])
{
    double speed = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double e[3] = {0.0, 0.0, 0.0};
    e[normal] = 1.0;
    double t[3] = {e[1] * n[2] - e[2] * n[1], e[2] * n[0] - e[0] * n[2], e[0] * n[1] - e[1] * n[0]};
    double st = 2.0 * u[0] - 1.0, ct = sqrt(1.0 - st * st);
    for (int a = 0; a < 3; ++a) v[a] = speed * (ct * n[a] + st * t[a]);
}

void or_scatter_uniforms(uint64_t seed, uint32_t p, uint32_t step, uint32_t sid, double u[2])
{
    uint32_t ctr[4] = {p, step, sid, 0x80000000u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    or_philox4x32_10(ctr, key, r);
    u[0] = or_u53(r[0], r[1]);
    u[1] = or_u53(r[2], r[3]);
}

/* Inward unit normal where a particle at X (cell units, outside its region)
 * left it: ball, -(X - c)/|X - c|; box, the normalised sum of the inward
 * normals of the faces it is beyond. */
static void inward_normal(const or_species* s, int dims, const double X[3], double n[3])
{
    n[0] = n[1] = n[2] = 0.0;
    if (s->region == OR_REGION_BALL) {
        for (int a = 0; a < dims; ++a) n[a] = s->rc[a] - X[a];
    } else {
        for (int a = 0; a < dims; ++a) {
            if (X[a] > s->rhi[a]) n[a] = -1.0;
            else if (X[a] < s->rlo[a]) n[a] = 1.0;
        }
    }
    double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int a = 0; a < 3; ++a) n[a] /= l;
}

/* ------------------------------------------------------------------------- */
/* Simulation state                                                          */
/* ------------------------------------------------------------------------- */
#define OR_MAX_SPECIES 8

/* Positions are carried as an integer cell index plus an offset in [0,1) along
 * each active axis (cell units), so that a step's move of 1e-6 cell or less is
 * not lost to the rounding of an absolute coordinate.  Bound particles keep
 * their anchor in C, O and their displacement in xi. */
typedef struct {
    or_species sp;
    size_t n;
    long* C;    /* [n][3] cell index (bound: anchor cell)                  */
    double* O;  /* [n][3] in-cell offset in [0,1) (bound: anchor offset)   */
    double* v;  /* [n][3] velocity v_{n-1/2} [m/s]                         */
    double* xi; /* [n][3] bound displacement from the anchor [m]           */
} sp_state;

struct or_sim {
    or_grid g;
    int L[3];        /* array extent per axis                                */
    size_t len;      /* L[0] L[1] L[2]                                       */
    double* E[3];
    double* B[3];
    double* J[3];    /* particle current of the last step, J^{n+1/2}         */
    double* einv[3]; /* inverse permittivity at the E_c nodes (NULL: unit)   */
    double* eoff[6]; /* off-diagonal inverse permittivity (a, b), a != b, at */
                     /* the E_a nodes, order 01 02 10 12 20 21 (NULL: none)  */
    double* eext[3]; /* static external field at the E_c nodes (NULL: none)  */
    double* rho_ion; /* fixed background charge density at nodes            */
    int have_ion;
    int nsp;
    sp_state sp[OR_MAX_SPECIES];
    long step;
    double* series;  /* [step][3] total particle current sum q w v_{n+1/2}  */
    size_t series_n, series_cap;
    int track;       /* 1: measure the continuity residual every step       */
    double cont_res, cont_scale;
    int ntile[3];
};

void or_track_continuity(or_sim* s, int on) { s->track = on; }

long or_steps_done(const or_sim* s) { return s->step; }

static int active(const or_sim* s, int a) { return a < s->g.dims; }
static int is_open(const or_sim* s, int a) { return active(s, a) && !s->g.periodic[a]; }

/* A component sits at a half-integer position along axis a if half[a] != 0.
 * Yee staggering (Sec. 4.1): E_x at (i+1/2, j, k), E_y at (i, j+1/2, k),
 * E_z at (i, j, k+1/2); B_x at (i, j+1/2, k+1/2), B_y at (i+1/2, j, k+1/2),
 * B_z at (i+1/2, j+1/2, k).  J sits with E, rho at the nodes. */
static void stag_E(int c, int half[3]) { for (int a = 0; a < 3; ++a) half[a] = (a == c); }
static void stag_B(int c, int half[3]) { for (int a = 0; a < 3; ++a) half[a] = (a != c); }

/* Number of valid entries of a component along axis a. */
static int valid_len(const or_sim* s, int a, int half)
{
    if (!active(s, a)) return 1;
    if (s->g.periodic[a]) return s->g.n[a];
    return half ? s->g.n[a] : s->g.n[a] + 1;
}

/* Flat index with periodic wrap; aborts on an index outside an open axis. */
static size_t fidx(const or_sim* s, long i, long j, long k)
{
    long ijk[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        if (!active(s, a)) { ijk[a] = 0; continue; }
        if (s->g.periodic[a]) {
            long n = s->g.n[a];
            ijk[a] = ((ijk[a] % n) + n) % n;
        } else if (ijk[a] < 0 || ijk[a] >= s->L[a]) {
            fprintf(stderr, "pic_oracle: grid index %ld out of range on axis %d\n", ijk[a], a);
            abort();
        }
    }
    return ((size_t)ijk[2] * (size_t)s->L[1] + (size_t)ijk[1]) * (size_t)s->L[0] + (size_t)ijk[0];
}

static double dvol(const or_sim* s)
{
    double v = 1.0;
    for (int a = 0; a < s->g.dims; ++a) v *= s->g.dx[a];
    return v;
}

int or_create(const or_grid* g, or_sim** out)
{
    if (!g || !out || g->dims < 1 || g->dims > 3 || g->dt <= 0.0 || g->sort_every < 1) return -1;
    or_sim* s = (or_sim*)calloc(1, sizeof(or_sim));
    if (!s) return -2;
    s->g = *g;
    s->len = 1;
    for (int a = 0; a < 3; ++a) {
        if (a >= g->dims) {
            s->g.n[a] = 1; s->g.periodic[a] = 1; s->g.tile[a] = 1;
            if (s->g.dx[a] <= 0.0) s->g.dx[a] = 1.0;
        }
        if (s->g.n[a] < 1 || s->g.tile[a] < 1 || s->g.dx[a] <= 0.0) { free(s); return -1; }
        s->L[a] = (a < g->dims && !g->periodic[a]) ? g->n[a] + 1 : s->g.n[a];
        s->len *= (size_t)s->L[a];
        s->ntile[a] = (s->g.n[a] + s->g.tile[a] - 1) / s->g.tile[a];
    }
    for (int c = 0; c < 3; ++c) {
        s->E[c] = (double*)calloc(s->len, sizeof(double));
        s->B[c] = (double*)calloc(s->len, sizeof(double));
        s->J[c] = (double*)calloc(s->len, sizeof(double));
        if (!s->E[c] || !s->B[c] || !s->J[c]) { or_destroy(s); return -2; }
    }
    s->rho_ion = (double*)calloc(s->len, sizeof(double));
    if (!s->rho_ion) { or_destroy(s); return -2; }
    *out = s;
    return 0;
}

void or_destroy(or_sim* s)
{
    if (!s) return;
    for (int c = 0; c < 3; ++c) {
        free(s->E[c]); free(s->B[c]); free(s->J[c]); free(s->einv[c]); free(s->eext[c]);
    }
    for (int m = 0; m < 6; ++m) free(s->eoff[m]);
    free(s->rho_ion);
    for (int i = 0; i < s->nsp; ++i) { free(s->sp[i].C); free(s->sp[i].O); free(s->sp[i].v); free(s->sp[i].xi); }
    free(s->series);
    free(s);
}

static int check_species(const or_sim* s, const or_species* sp)
{
    if (sp->kind < OR_FREE || sp->kind > OR_DIRAC || sp->m <= 0.0) return -1;
    if (sp->reflect < 0 || sp->reflect > 2) return -1;
    /* diffusive draws: free carriers (3D) and Dirac carriers with a sheet normal (in-sheet) */
    if (sp->reflect == 2 && !(sp->kind == OR_FREE || (sp->kind == OR_DIRAC && sp->sheet_normal >= 0))) return -1;
    if (sp->mass_per_particle && sp->kind != OR_DIRAC) return -1;
    if (sp->region == OR_REGION_BALL)
        for (int a = 1; a < s->g.dims; ++a)
            if (s->g.dx[a] != s->g.dx[0]) return -1;
    return 0;
}

static double* dup3(const double* src, size_t n, double scale0, double scale1, double scale2)
{
    double* d = (double*)malloc(sizeof(double) * 3 * (n ? n : 1));
    if (!d) return NULL;
    for (size_t i = 0; i < n; ++i) {
        d[3 * i + 0] = src ? src[3 * i + 0] * scale0 : 0.0;
        d[3 * i + 1] = src ? src[3 * i + 1] * scale1 : 0.0;
        d[3 * i + 2] = src ? src[3 * i + 2] * scale2 : 0.0;
    }
    return d;
}

/* Renormalise a position to offset in [0,1) and wrap the cell on periodic axes. */
static void normalize(const or_sim* s, long C[3], double O[3])
{
    for (int a = 0; a < s->g.dims; ++a) {
        double f = floor(O[a]);
        C[a] += (long)f;
        O[a] -= f;
        if (O[a] >= 1.0) { O[a] = 0.0; C[a] += 1; }
        if (s->g.periodic[a]) {
            long n = s->g.n[a];
            C[a] = ((C[a] % n) + n) % n;
        }
    }
}

/* Cell and offset of an absolute position X (cell units). */
static void set_position(const or_sim* s, const double X[3], long C[3], double O[3])
{
    for (int a = 0; a < 3; ++a) { C[a] = 0; O[a] = 0.0; }
    for (int a = 0; a < s->g.dims; ++a) O[a] = X[a];
    normalize(s, C, O);
}

int or_add_species(or_sim* s, const or_species* sp, size_t n,
                   const double* x, const double* v, const double* xi)
{
    if (!s || !sp || s->nsp >= OR_MAX_SPECIES || check_species(s, sp)) return -1;
    sp_state* st = &s->sp[s->nsp];
    st->sp = *sp;
    st->n = n;
    st->C = (long*)calloc(3 * (n ? n : 1), sizeof(long));
    st->O = (double*)calloc(3 * (n ? n : 1), sizeof(double));
    st->v = dup3(v, n, 1.0, 1.0, 1.0);
    /* bound: displacements; Dirac with per-particle mass: m_d in xi[i][0] */
    int keep = sp->kind == OR_BOUND || (sp->kind == OR_DIRAC && sp->mass_per_particle);
    st->xi = dup3(keep ? xi : NULL, n, 1.0, 1.0, 1.0);
    if (!st->C || !st->O || !st->v || !st->xi) return -2;
    if (sp->kind == OR_DIRAC && sp->mass_per_particle)
        for (size_t i = 0; i < n; ++i)
            if (!(st->xi[3 * i] > 0.0)) return -1;
    for (size_t i = 0; i < n; ++i) {
        double X[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < s->g.dims; ++a) X[a] = x[3 * i + a] / s->g.dx[a];
        set_position(s, X, &st->C[3 * i], &st->O[3 * i]);
    }
    return s->nsp++;
}

/* Cells of a region, in row-major order (x fastest).  A cell belongs to a
 * ball if all its corners are within the radius, to a box if it lies inside
 * the box (cell units). */
static int cell_in_region(const or_sim* s, const or_species* sp, const int c[3])
{
    int d = s->g.dims;
    if (sp->region == OR_REGION_ALL) return 1;
    if (sp->region == OR_REGION_BOX) {
        for (int a = 0; a < d; ++a)
            if ((double)c[a] < sp->rlo[a] || (double)(c[a] + 1) > sp->rhi[a]) return 0;
        return 1;
    }
    for (int corner = 0; corner < (1 << d); ++corner) {
        double r2 = 0.0;
        for (int a = 0; a < d; ++a) {
            double p = (double)(c[a] + ((corner >> a) & 1)) - sp->rc[a];
            r2 += p * p;
        }
        if (r2 > sp->rr * sp->rr) return 0;
    }
    return 1;
}

/* Module I: species loader (Sec. 2).  Free species draw speeds from the FD
 * distribution eq:fddist with an isotropic direction; Dirac carriers draw only
 * an in-sheet direction (their speed is v_F and their mass fixed, Sec. 5);
 * bound particles start at rest with a displacement uniform in a small ball.
 * Positions are uniform in each region cell (or, in 1D, a quiet start with a
 * Lagrangian sine displacement).  The density comes from E_F when not given.
 * Random numbers: six uniforms per particle from Philox (draw6). */
int or_init_species(or_sim* s, const or_species* spin, const or_init* ini, int* sid_out)
{
    if (!s || !spin || !ini || ini->ppc < 1 || check_species(s, spin)) return -1;
    if (ini->loading == OR_LOAD_QUIET && s->g.dims != 1) return -1;
    if (s->nsp >= OR_MAX_SPECIES) return -1;
    or_species sp = *spin;
    int sid = s->nsp;
    int d = s->g.dims;

    /* region cells */
    size_t ncell = 0;
    int c[3];
    for (c[2] = 0; c[2] < s->g.n[2]; ++c[2])
        for (c[1] = 0; c[1] < s->g.n[1]; ++c[1])
            for (c[0] = 0; c[0] < s->g.n[0]; ++c[0])
                ncell += (size_t)cell_in_region(s, &sp, c);
    int* cells = (int*)malloc(sizeof(int) * 3 * (ncell ? ncell : 1));
    if (!cells) return -2;
    size_t q = 0;
    for (c[2] = 0; c[2] < s->g.n[2]; ++c[2])
        for (c[1] = 0; c[1] < s->g.n[1]; ++c[1])
            for (c[0] = 0; c[0] < s->g.n[0]; ++c[0])
                if (cell_in_region(s, &sp, c)) {
                    cells[3 * q] = c[0]; cells[3 * q + 1] = c[1]; cells[3 * q + 2] = c[2];
                    ++q;
                }

    double density = ini->density;
    if (density <= 0.0) {
        if (sp.kind == OR_DIRAC) density = or_dirac_density2d(ini->e_fermi, sp.v_f) /
                                           s->g.dx[sp.sheet_normal >= 0 ? sp.sheet_normal : 0];
        else density = or_density_from_fermi(ini->e_fermi, sp.m);
    }
    sp.weight = density * dvol(s) / (double)ini->ppc;

    size_t n = ncell * (size_t)ini->ppc;
    sp_state* st = &s->sp[sid];
    st->sp = sp;
    st->n = n;
    st->C = (long*)calloc(3 * (n ? n : 1), sizeof(long));
    st->O = (double*)calloc(3 * (n ? n : 1), sizeof(double));
    st->v = (double*)calloc(3 * (n ? n : 1), sizeof(double));
    st->xi = (double*)calloc(3 * (n ? n : 1), sizeof(double));
    if (!st->C || !st->O || !st->v || !st->xi) { free(cells); return -2; }

    double kT = KB * ini->temperature;
    fd_table* tab = NULL;
    const int dirac_mpp = sp.kind == OR_DIRAC && sp.mass_per_particle;
    if (((sp.kind == OR_FREE && ini->momentum == OR_MOM_FD) || dirac_mpp) && kT > 0.0) {
        tab = (fd_table*)malloc(sizeof(fd_table));
        if (!tab) { free(cells); return -2; }
        fd_table_build(tab, ini->e_fermi, kT, sp.kind == OR_DIRAC);
    }

    for (size_t p = 0; p < n; ++p) {
        size_t cr = p / (size_t)ini->ppc;
        int k = (int)(p % (size_t)ini->ppc);
        double u[6];
        draw6(ini->seed, sid, (uint64_t)p, u);
        long* Cp = &st->C[3 * p];
        double* Op = &st->O[3 * p];
        double* v = &st->v[3 * p];
        for (int a = 0; a < d; ++a) { Cp[a] = cells[3 * cr + a]; Op[a] = u[a]; }
        if (ini->loading == OR_LOAD_QUIET) {
            double x0 = (double)cells[3 * cr] + ((double)k + 0.5) / (double)ini->ppc;
            double nx = (double)s->g.n[0];
            double kw = 2.0 * PI * (double)ini->pert_mode / nx; /* per cell */
            double X[3] = {x0 + (ini->pert_amp / kw) * sin(kw * x0), 0.0, 0.0};
            set_position(s, X, Cp, Op);
        }
        if (sp.kind == OR_FREE) {
            if (ini->momentum == OR_MOM_FD) {
                double speed = fd_speed(tab, ini->e_fermi, kT, sp.m, u[3]);
                double ct = 2.0 * u[4] - 1.0;
                double st_ = sqrt(1.0 - ct * ct);
                double ph = 2.0 * PI * u[5];
                v[0] = speed * st_ * cos(ph);
                v[1] = speed * st_ * sin(ph);
                v[2] = speed * ct;
            }
        } else if (sp.kind == OR_DIRAC) {
            int e1 = -1, e2 = -1;
            for (int a = 0; a < 3; ++a) {
                if (a == sp.sheet_normal) continue;
                if (e1 < 0) e1 = a; else if (e2 < 0) e2 = a;
            }
            double ph = 2.0 * PI * u[3];
            v[e1] = sp.v_f * cos(ph);
            v[e2] = sp.v_f * sin(ph);
            /* Sec. 5: transverse mass m_d = p / v_F of this carrier, p = e / v_F, with its
             * energy e drawn from the 2D Fermi-Dirac distribution (u[4]) */
            if (dirac_mpp) {
                double e = dirac_energy(tab, ini->e_fermi, kT, u[4]);
                st->xi[3 * p + 0] = e / (sp.v_f * sp.v_f);
            }
        } else { /* bound */
            double r = ini->xi_radius * cbrt(u[3]);
            double ct = 2.0 * u[4] - 1.0;
            double st_ = sqrt(1.0 - ct * ct);
            double ph = 2.0 * PI * u[5];
            st->xi[3 * p + 0] = r * st_ * cos(ph);
            st->xi[3 * p + 1] = r * st_ * sin(ph);
            st->xi[3 * p + 2] = r * ct;
        }
    }
    free(tab);
    free(cells);
    s->nsp++;
    if (sid_out) *sid_out = sid;
    return 0;
}

double or_species_weight(const or_sim* s, int sid)
{
    return (sid >= 0 && sid < s->nsp) ? s->sp[sid].sp.weight : NAN;
}

size_t or_count(const or_sim* s, int sid)
{
    return (sid >= 0 && sid < s->nsp) ? s->sp[sid].n : 0;
}

int or_get_particles(const or_sim* s, int sid, double* x, double* v, double* xi)
{
    if (sid < 0 || sid >= s->nsp) return -1;
    const sp_state* st = &s->sp[sid];
    for (size_t i = 0; i < st->n; ++i)
        for (int a = 0; a < 3; ++a) {
            if (x) x[3 * i + a] = a < s->g.dims ? ((double)st->C[3 * i + a] + st->O[3 * i + a]) * s->g.dx[a] : 0.0;
            if (v) v[3 * i + a] = st->v[3 * i + a];
            if (xi) xi[3 * i + a] = st->xi[3 * i + a];
        }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Cell key and stable sort.  Reading: the paper does not sort; the key is    */
/* the tile-major linear cell index (tile id, then cell within the tile,     */
/* x fastest) so that a tile's particles are contiguous.  Bound particles are */
/* keyed on their anchor cell.                                               */
/* ------------------------------------------------------------------------- */
static int32_t cell_key(const or_sim* s, const int c[3])
{
    const int* T = s->g.tile;
    long tid = ((long)(c[2] / T[2]) * s->ntile[1] + (c[1] / T[1])) * s->ntile[0] + (c[0] / T[0]);
    long loc = ((long)(c[2] % T[2]) * T[1] + (c[1] % T[1])) * T[0] + (c[0] % T[0]);
    return (int32_t)(tid * (long)T[0] * T[1] * T[2] + loc);
}

static int32_t particle_key(const or_sim* s, const long C[3])
{
    int c[3] = {0, 0, 0};
    for (int a = 0; a < s->g.dims; ++a) {
        c[a] = (int)C[a];
        if (c[a] < 0) c[a] = 0;
        if (c[a] >= s->g.n[a]) c[a] = s->g.n[a] - 1;
    }
    return cell_key(s, c);
}

int or_keys(const or_sim* s, int sid, int32_t* keys)
{
    if (sid < 0 || sid >= s->nsp) return -1;
    const sp_state* st = &s->sp[sid];
    for (size_t i = 0; i < st->n; ++i) keys[i] = particle_key(s, &st->C[3 * i]);
    return 0;
}

/* Stable counting sort by key. */
static int sort_species(or_sim* s, sp_state* st)
{
    size_t n = st->n;
    if (n == 0) return 0;
    long nkeys = (long)s->ntile[0] * s->ntile[1] * s->ntile[2] *
                 (long)s->g.tile[0] * s->g.tile[1] * s->g.tile[2];
    size_t* count = (size_t*)calloc((size_t)nkeys + 1, sizeof(size_t));
    int32_t* key = (int32_t*)malloc(sizeof(int32_t) * n);
    size_t* perm = (size_t*)malloc(sizeof(size_t) * n);
    double* tmp = (double*)malloc(sizeof(double) * 3 * n);
    long* tmpc = (long*)malloc(sizeof(long) * 3 * n);
    if (!count || !key || !perm || !tmp || !tmpc) {
        free(count); free(key); free(perm); free(tmp); free(tmpc);
        return -2;
    }
    for (size_t i = 0; i < n; ++i) {
        key[i] = particle_key(s, &st->C[3 * i]);
        count[key[i] + 1]++;
    }
    for (long k = 0; k < nkeys; ++k) count[k + 1] += count[k];
    for (size_t i = 0; i < n; ++i) perm[count[key[i]]++] = i;
    double* arrs[3] = {st->O, st->v, st->xi};
    for (int w = 0; w < 3; ++w) {
        for (size_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) tmp[3 * i + a] = arrs[w][3 * perm[i] + a];
        memcpy(arrs[w], tmp, sizeof(double) * 3 * n);
    }
    for (size_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) tmpc[3 * i + a] = st->C[3 * perm[i] + a];
    memcpy(st->C, tmpc, sizeof(long) * 3 * n);
    free(count); free(key); free(perm); free(tmp); free(tmpc);
    return 0;
}

int or_sort(or_sim* s)
{
    for (int i = 0; i < s->nsp; ++i) {
        int r = sort_species(s, &s->sp[i]);
        if (r) return r;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Field gather (Appendix A.1: E_n, B_n interpolated to the particle).        */
/* Reading: first-order (cloud-in-cell) weights on each component's own      */
/* staggered location.                                                       */
/* ------------------------------------------------------------------------- */
static double gather(const or_sim* s, const double* F, const int half[3], const long C[3], const double O[3])
{
    long base[3] = {0, 0, 0};
    double w1[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < s->g.dims; ++a) {
        double u = O[a] - (half[a] ? 0.5 : 0.0);
        double f = floor(u);
        base[a] = C[a] + (long)f;
        w1[a] = u - f;
    }
    double sum = 0.0;
    int na[3] = {1, 1, 1};
    for (int a = 0; a < s->g.dims; ++a) na[a] = 2;
    for (int dk = 0; dk < na[2]; ++dk)
        for (int dj = 0; dj < na[1]; ++dj)
            for (int di = 0; di < na[0]; ++di) {
                int dd[3] = {di, dj, dk};
                double w = 1.0;
                for (int a = 0; a < s->g.dims; ++a) w *= dd[a] ? w1[a] : (1.0 - w1[a]);
                sum += w * F[fidx(s, base[0] + di, base[1] + dj, base[2] + dk)];
            }
    return sum;
}

/* The particles feel E + E_ext: the static external (work-function) field of Sec. 3 sits on the
 * E nodes, is gathered like E and never enters the Maxwell update. */
static void gather_EB(const or_sim* s, const long C[3], const double O[3], double E[3], double B[3])
{
    int h[3];
    for (int c = 0; c < 3; ++c) {
        stag_E(c, h); E[c] = gather(s, s->E[c], h, C, O);
        if (s->eext[c]) E[c] += gather(s, s->eext[c], h, C, O);
        stag_B(c, h); B[c] = gather(s, s->B[c], h, C, O);
    }
}

/* Fields at a point x (metres), for tests. */
int or_gather_at(const or_sim* s, const double x[3], double E[3], double B[3])
{
    double X[3] = {0.0, 0.0, 0.0}, O[3];
    long C[3];
    for (int a = 0; a < s->g.dims; ++a) X[a] = x[a] / s->g.dx[a];
    set_position(s, X, C, O);
    gather_EB(s, C, O, E, B);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Charge-conserving current deposition.  The paper deposits J_f from the    */
/* macroparticles (eq:consteps) without naming the scheme.  Reading:          */
/* Esirkepov (Comput. Phys. Commun. 135, 144 (2001)) with first-order shapes  */
/* S(x) = max(0, 1 - |x|) along the straight segment from x0 to x1, both      */
/* given relative to the start cell c0 (cell units).  Reading: the move is    */
/* the push displacement dt v_{n+1/2} (eq:discrvel, and xi_{n+1} - xi_n for a */
/* bound particle), added to the start offset, so it is not recomputed as a   */
/* difference of rounded absolute positions.                                  */
/* ------------------------------------------------------------------------- */
static double shape1(double x) { double a = fabs(x); return a < 1.0 ? 1.0 - a : 0.0; }

static void deposit(or_sim* s, double qw, const long c0[3], const double x0[3], const double x1[3],
                    const double v[3])
{
    int d = s->g.dims;
    const double* dx = s->g.dx;
    const double dt = s->g.dt;
    double S0[3][4], S1[3][4], DS[3][4];
    for (int a = 0; a < 3; ++a)
        for (int m = 0; m < 4; ++m) { S0[a][m] = S1[a][m] = DS[a][m] = 0.0; }
    for (int a = 0; a < d; ++a) {
        if (fabs(x1[a] - x0[a]) >= 1.0) {
            fprintf(stderr, "pic_oracle: displacement of a cell or more in one step\n");
            abort();
        }
        for (int m = 0; m < 4; ++m) {
            double node = (double)(m - 1);
            S0[a][m] = shape1(x0[a] - node);
            S1[a][m] = shape1(x1[a] - node);
            DS[a][m] = S1[a][m] - S0[a][m];
        }
    }
    if (d == 1) {
        /* J_x(i+1/2) = -(q w / dt) sum_{i' <= i} DS(i');
         * J_y, J_z(i) = q w v_{y,z} (S0 + S1)(i) / (2 dx). */
        double run = 0.0;
        for (int m = 0; m < 4; ++m) {
            run += DS[0][m];
            long i = c0[0] + m - 1;
            s->J[0][fidx(s, i, 0, 0)] += -qw / dt * run;
            s->J[1][fidx(s, i, 0, 0)] += qw * v[1] * 0.5 * (S0[0][m] + S1[0][m]) / dx[0];
            s->J[2][fidx(s, i, 0, 0)] += qw * v[2] * 0.5 * (S0[0][m] + S1[0][m]) / dx[0];
        }
    } else if (d == 2) {
        /* W_x = DS_x (S0_y + DS_y / 2), W_y = DS_y (S0_x + DS_x / 2);
         * J_x(i+1/2, j) = -(q w / (dt dy)) sum_{i'<=i} W_x(i', j), and
         * likewise J_y; J_z(i, j) = q w v_z / (dx dy) *
         * [S0x S0y + (DSx S0y + S0x DSy)/2 + DSx DSy / 3]. */
        for (int mj = 0; mj < 4; ++mj) {
            double run = 0.0;
            for (int mi = 0; mi < 4; ++mi) {
                run += DS[0][mi] * (S0[1][mj] + 0.5 * DS[1][mj]);
                s->J[0][fidx(s, c0[0] + mi - 1, c0[1] + mj - 1, 0)] += -qw / (dt * dx[1]) * run;
            }
        }
        for (int mi = 0; mi < 4; ++mi) {
            double run = 0.0;
            for (int mj = 0; mj < 4; ++mj) {
                run += DS[1][mj] * (S0[0][mi] + 0.5 * DS[0][mi]);
                s->J[1][fidx(s, c0[0] + mi - 1, c0[1] + mj - 1, 0)] += -qw / (dt * dx[0]) * run;
            }
        }
        for (int mj = 0; mj < 4; ++mj)
            for (int mi = 0; mi < 4; ++mi) {
                double wz = S0[0][mi] * S0[1][mj] + 0.5 * (DS[0][mi] * S0[1][mj] + S0[0][mi] * DS[1][mj]) +
                            DS[0][mi] * DS[1][mj] / 3.0;
                s->J[2][fidx(s, c0[0] + mi - 1, c0[1] + mj - 1, 0)] += qw * v[2] / (dx[0] * dx[1]) * wz;
            }
    } else {
        /* W_x = DS_x [S0_y S0_z + DS_y S0_z / 2 + S0_y DS_z / 2 + DS_y DS_z / 3]
         * (and cyclic); J_x(i+1/2, j, k) = -(q w / (dt dy dz)) sum_{i'<=i} W_x. */
        for (int axis = 0; axis < 3; ++axis) {
            int a1 = (axis + 1) % 3, a2 = (axis + 2) % 3;
            double pref = -qw / (dt * dx[a1] * dx[a2]);
            for (int m2 = 0; m2 < 4; ++m2)
                for (int m1 = 0; m1 < 4; ++m1) {
                    double t = S0[a1][m1] * S0[a2][m2] + 0.5 * DS[a1][m1] * S0[a2][m2] +
                               0.5 * S0[a1][m1] * DS[a2][m2] + DS[a1][m1] * DS[a2][m2] / 3.0;
                    double run = 0.0;
                    for (int m0 = 0; m0 < 4; ++m0) {
                        run += DS[axis][m0] * t;
                        long ijk[3];
                        ijk[axis] = c0[axis] + m0 - 1;
                        ijk[a1] = c0[a1] + m1 - 1;
                        ijk[a2] = c0[a2] + m2 - 1;
                        s->J[axis][fidx(s, ijk[0], ijk[1], ijk[2])] += pref * run;
                    }
                }
        }
    }
}

/* Charge density at the nodes with first-order shapes: rho = q w prod S / dV. */
static void deposit_rho(const or_sim* s, double* rho)
{
    memset(rho, 0, sizeof(double) * s->len);
    double dv = dvol(s);
    int d = s->g.dims;
    for (int i = 0; i < s->nsp; ++i) {
        const sp_state* st = &s->sp[i];
        double qw = st->sp.q * st->sp.weight;
        for (size_t p = 0; p < st->n; ++p) {
            long b[3] = {0, 0, 0};
            double w1[3] = {0, 0, 0};
            for (int a = 0; a < d; ++a) {
                double r = st->O[3 * p + a] + (st->sp.kind == OR_BOUND ? st->xi[3 * p + a] / s->g.dx[a] : 0.0);
                double f = floor(r);
                b[a] = st->C[3 * p + a] + (long)f;
                w1[a] = r - f;
            }
            int na[3] = {1, 1, 1};
            for (int a = 0; a < d; ++a) na[a] = 2;
            for (int dk = 0; dk < na[2]; ++dk)
                for (int dj = 0; dj < na[1]; ++dj)
                    for (int di = 0; di < na[0]; ++di) {
                        int dd[3] = {di, dj, dk};
                        double w = 1.0;
                        for (int a = 0; a < d; ++a) w *= dd[a] ? w1[a] : (1.0 - w1[a]);
                        rho[fidx(s, b[0] + di, b[1] + dj, b[2] + dk)] += qw * w / dv;
                    }
        }
    }
}

int or_get_rho(const or_sim* s, double* rho)
{
    deposit_rho(s, rho);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Yee field update (Sec. 4.1 and eq:consteps with a unit dielectric tensor). */
/* Readings: SI form dE/dt = c^2 curl B - J / eps0, dB/dt = -curl E (the      */
/* printed c dt and mu0 J mix unit systems); J is J^{n+1/2} deposited from    */
/* x_n to x_{n+1}; B, which Yee keeps at half steps, is advanced in two       */
/* half steps around the E update so that the push sees B_n.  Open faces use  */
/* first-order Mur boundaries on the tangential E.                            */
/* ------------------------------------------------------------------------- */
static double dfwd(const or_sim* s, const double* F, long i, long j, long k, int a)
{
    if (!active(s, a)) return 0.0;
    long e[3] = {0, 0, 0};
    e[a] = 1;
    return (F[fidx(s, i + e[0], j + e[1], k + e[2])] - F[fidx(s, i, j, k)]) / s->g.dx[a];
}

static double dbwd(const or_sim* s, const double* F, long i, long j, long k, int a)
{
    if (!active(s, a)) return 0.0;
    long e[3] = {0, 0, 0};
    e[a] = 1;
    return (F[fidx(s, i, j, k)] - F[fidx(s, i - e[0], j - e[1], k - e[2])]) / s->g.dx[a];
}

static void b_half_step(or_sim* s)
{
    double h = 0.5 * s->g.dt;
    for (int c = 0; c < 3; ++c) {
        int half[3];
        stag_B(c, half);
        int n0 = valid_len(s, 0, half[0]), n1 = valid_len(s, 1, half[1]), n2 = valid_len(s, 2, half[2]);
        int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        for (long k = 0; k < n2; ++k)
            for (long j = 0; j < n1; ++j)
                for (long i = 0; i < n0; ++i) {
                    /* (curl E)_c = d_{a1} E_{a2} - d_{a2} E_{a1} */
                    double curl = dfwd(s, s->E[a2], i, j, k, a1) - dfwd(s, s->E[a1], i, j, k, a2);
                    s->B[c][fidx(s, i, j, k)] -= h * curl;
                }
    }
}

/* Axis on whose open face an E_c node sits (lowest such axis), or -1. */
static int mur_axis(const or_sim* s, int c, const long ijk[3])
{
    for (int a = 0; a < 3; ++a) {
        if (a == c || !is_open(s, a)) continue;
        if (ijk[a] == 0 || ijk[a] == s->g.n[a]) return a;
    }
    return -1;
}

static double source_value(const or_sim* s, double t)
{
    const or_grid* g = &s->g;
    if (g->src_kind == OR_SRC_NONE || t < 0.0 || t > g->src_tau) return 0.0;
    double env = sin(PI * t / g->src_tau);
    return g->src_j0 * env * env * sin(g->src_omega * t);
}

static int source_hits(const or_sim* s, int c, const long ijk[3])
{
    const or_grid* g = &s->g;
    if (g->src_kind == OR_SRC_NONE || c != g->src_comp) return 0;
    if (g->src_kind == OR_SRC_SHEET) return ijk[g->src_axis] == g->src_index[g->src_axis];
    for (int a = 0; a < 3; ++a)
        if (active(s, a) && ijk[a] != g->src_index[a]) return 0;
    return 1;
}

/* Off-diagonal slot of the pair (a, b), a != b: order 01 02 10 12 20 21. */
static int off_slot(int a, int b) { return 2 * a + (b > a ? b - 1 : b); }

/* The mean of U_b over the E_b nodes nearest to the E_a node ijk.  The two
 * sit half a cell apart along a and along b (E_a is half-integer along a,
 * E_b along b), so the nearest E_b nodes are ijk + s e_a - t e_b with s, t in
 * {0, 1} on the active axes: four in 2D and 3D when both axes are active, two
 * when one is, one when neither is. */
static double mean_nearest(const or_sim* s, const double* Ub, int a, int b, const long ijk[3])
{
    int ns = active(s, a) ? 2 : 1, nt = active(s, b) ? 2 : 1;
    double sum = 0.0;
    for (int sa = 0; sa < ns; ++sa)
        for (int tb = 0; tb < nt; ++tb) {
            long h[3] = {ijk[0], ijk[1], ijk[2]};
            h[a] += sa;
            h[b] -= tb;
            sum += Ub[fidx(s, h[0], h[1], h[2])];
        }
    return sum / (double)(ns * nt);
}

static void e_step(or_sim* s, double t_half)
{
    double dt = s->g.dt, c2 = CLIGHT * CLIGHT;
    double jsrc = source_value(s, t_half);
    double* Eold[3];
    double* Emid[3];
    double* U[3] = {NULL, NULL, NULL};
    int tensor = 0;
    for (int m = 0; m < 6; ++m)
        if (s->eoff[m]) tensor = 1;
    for (int c = 0; c < 3; ++c) {
        Eold[c] = (double*)malloc(sizeof(double) * s->len);
        memcpy(Eold[c], s->E[c], sizeof(double) * s->len);
        if (tensor) U[c] = (double*)calloc(s->len, sizeof(double));
    }
    for (int c = 0; c < 3; ++c) {
        int half[3];
        stag_E(c, half);
        int n0 = valid_len(s, 0, half[0]), n1 = valid_len(s, 1, half[1]), n2 = valid_len(s, 2, half[2]);
        int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        for (long k = 0; k < n2; ++k)
            for (long j = 0; j < n1; ++j)
                for (long i = 0; i < n0; ++i) {
                    long ijk[3] = {i, j, k};
                    if (mur_axis(s, c, ijk) >= 0) continue;
                    double curl = dbwd(s, s->B[a2], i, j, k, a1) - dbwd(s, s->B[a1], i, j, k, a2);
                    double jc = s->J[c][fidx(s, i, j, k)] + (source_hits(s, c, ijk) ? jsrc : 0.0);
                    /* eq:consteps: the curl and current terms are scaled by the inverse
                     * dielectric tensor; its diagonal entry is taken at the E_c node */
                    double ei = s->einv[c] ? s->einv[c][fidx(s, i, j, k)] : 1.0;
                    double u = c2 * curl - jc / EPS0;
                    if (tensor) U[c][fidx(s, i, j, k)] = u;
                    s->E[c][fidx(s, i, j, k)] += dt * ei * u;
                }
    }
    /* eq:consteps with a full tensor: row a of the inverse tensor at the E_a node
     * multiplies the update vector, whose other components live on their own
     * nodes and are averaged onto the E_a node (mean_nearest).  Off-diagonal
     * entries are nonzero only two nodes or more inside every open face, so the
     * averaged nodes are interior nodes with a computed U. */
    if (tensor)
        for (int a = 0; a < 3; ++a) {
            int half[3];
            stag_E(a, half);
            int n0 = valid_len(s, 0, half[0]), n1 = valid_len(s, 1, half[1]), n2 = valid_len(s, 2, half[2]);
            for (long k = 0; k < n2; ++k)
                for (long j = 0; j < n1; ++j)
                    for (long i = 0; i < n0; ++i) {
                        long ijk[3] = {i, j, k};
                        size_t q = fidx(s, i, j, k);
                        double sum = 0.0;
                        int any = 0;
                        for (int b = 0; b < 3; ++b) {
                            if (b == a || !s->eoff[off_slot(a, b)]) continue;
                            double o = s->eoff[off_slot(a, b)][q];
                            if (o == 0.0) continue;
                            sum += o * mean_nearest(s, U[b], a, b, ijk);
                            any = 1;
                        }
                        if (any) s->E[a][q] += dt * sum;
                    }
        }
    for (int c = 0; c < 3; ++c) {
        Emid[c] = (double*)malloc(sizeof(double) * s->len);
        memcpy(Emid[c], s->E[c], sizeof(double) * s->len);
    }
    /* Mur (1981), first order: E^{n+1}_b = E^n_{b'} + k (E^{n+1}_{b'} - E^n_b),
     * b' the inward neighbour, k = (c dt - dx) / (c dt + dx).  The inward
     * value is the one after the curl update (at an edge, where the inward
     * neighbour is itself on a face, that is its old value).
     * Reading: the faces absorb at the vacuum speed c; the inverse permittivity
     * is not used on face nodes (media end before the open faces). */
    for (int c = 0; c < 3; ++c) {
        int half[3];
        stag_E(c, half);
        int n0 = valid_len(s, 0, half[0]), n1 = valid_len(s, 1, half[1]), n2 = valid_len(s, 2, half[2]);
        for (long k = 0; k < n2; ++k)
            for (long j = 0; j < n1; ++j)
                for (long i = 0; i < n0; ++i) {
                    long ijk[3] = {i, j, k};
                    int a = mur_axis(s, c, ijk);
                    if (a < 0) continue;
                    long in[3] = {i, j, k};
                    in[a] += (ijk[a] == 0) ? 1 : -1;
                    double kc = (CLIGHT * dt - s->g.dx[a]) / (CLIGHT * dt + s->g.dx[a]);
                    size_t b = fidx(s, i, j, k), bi = fidx(s, in[0], in[1], in[2]);
                    s->E[c][b] = Eold[c][bi] + kc * (Emid[c][bi] - Eold[c][b]);
                }
    }
    for (int c = 0; c < 3; ++c) { free(Eold[c]); free(Emid[c]); free(U[c]); }
}

/* ------------------------------------------------------------------------- */
/* One PIC cycle per step (Appendix A.1 and Sec. 4.1): gather E_n, B_n at x_n; */
/* push to v_{n+1/2}, x_{n+1}; material boundary; deposit J^{n+1/2};           */
/* B_{n+1/2}, E_{n+1}, B_{n+1}.                                               */
/* ------------------------------------------------------------------------- */
static int series_push(or_sim* s, const double I[3])
{
    if (s->series_n == s->series_cap) {
        size_t cap = s->series_cap ? 2 * s->series_cap : 1024;
        double* p = (double*)realloc(s->series, sizeof(double) * 3 * cap);
        if (!p) return -2;
        s->series = p;
        s->series_cap = cap;
    }
    memcpy(&s->series[3 * s->series_n], I, sizeof(double) * 3);
    s->series_n++;
    return 0;
}

static void particle_step(or_sim* s, double I[3])
{
    int d = s->g.dims;
    double dt = s->g.dt;
    I[0] = I[1] = I[2] = 0.0;
    for (int c = 0; c < 3; ++c) memset(s->J[c], 0, sizeof(double) * s->len);
    for (int isp = 0; isp < s->nsp; ++isp) {
        sp_state* st = &s->sp[isp];
        const or_species* sp = &st->sp;
        double qm = sp->q / sp->m, qw = sp->q * sp->weight;
        for (size_t p = 0; p < st->n; ++p) {
            long* Cp = &st->C[3 * p];
            double* Op = &st->O[3 * p];
            double* v = &st->v[3 * p];
            double* xi = &st->xi[3 * p];
            long c0[3] = {0, 0, 0};
            double x0[3] = {0.0, 0.0, 0.0}, x1[3] = {0.0, 0.0, 0.0}, E[3], B[3];
            /* start cell and offset of x_n (bound: anchor plus displacement) */
            for (int a = 0; a < d; ++a) {
                double r = Op[a] + (sp->kind == OR_BOUND ? xi[a] / s->g.dx[a] : 0.0);
                double f = floor(r);
                c0[a] = Cp[a] + (long)f;
                x0[a] = r - f;
                if (x0[a] >= 1.0) { x0[a] = 0.0; c0[a] += 1; }
            }
            gather_EB(s, c0, x0, E, B);
            if (sp->kind == OR_FREE) or_push_free(qm, dt, E, B, v);
            else if (sp->kind == OR_BOUND)
                or_push_bound(qm, dt, sp->omega0_sq, sp->gamma, sp->b_weight, E, B, xi, v);
            else {
                /* Sec. 5: the per-particle transverse mass, when the species carries one */
                double qmd = sp->mass_per_particle ? sp->q / xi[0] : qm;
                or_push_dirac(qmd, dt, sp->v_f, sp->sheet_normal, E, B, v);
            }
            /* x_{n+1} = x_n + dt v_{n+1/2} (eq:discrvel; xi_{n+1} = xi_n + dt v for bound particles) */
            for (int a = 0; a < d; ++a) x1[a] = x0[a] + dt * v[a] / s->g.dx[a];
            if (sp->kind == OR_BOUND) {
                for (int a = 0; a < 3; ++a) xi[a] = xi[a] + dt * v[a];
            } else if (sp->reflect) {
                double X[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < d; ++a) X[a] = (double)c0[a] + x1[a];
                double n[3];
                if (sp->reflect == 2) inward_normal(sp, d, X, n);  /* at the escaped point */
                if (or_reflect(sp, d, X, v)) {
                    for (int a = 0; a < d; ++a) x1[a] = X[a] - (double)c0[a];
                    if (sp->reflect == 2) {
                        double u[2];
                        or_scatter_uniforms(sp->seed, (uint32_t)p, (uint32_t)s->step, (uint32_t)isp, u);
                        if (sp->kind == OR_DIRAC) {
                            /* the in-sheet part of the normal, renormalised; where it vanishes
                             * (a crossing along the sheet normal, which an in-sheet carrier does
                             * not make) the specular result stands */
                            n[sp->sheet_normal] = 0.0;
                            double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
                            if (l > 0.0) {
                                for (int a = 0; a < 3; ++a) n[a] /= l;
                                or_lambert2d(n, sp->sheet_normal, u, v);
                            }
                        } else {
                            or_lambert(n, u, v);
                        }
                    }
                }
            }
            deposit(s, qw, c0, x0, x1, v);
            for (int a = 0; a < 3; ++a) I[a] += qw * v[a];
            if (sp->kind != OR_BOUND) {
                for (int a = 0; a < d; ++a) { Cp[a] = c0[a]; Op[a] = x1[a]; }
                normalize(s, Cp, Op);
            }
        }
    }
}

int or_step(or_sim* s, int nsteps)
{
    if (!s || nsteps < 0) return -1;
    double* rho0 = (double*)malloc(sizeof(double) * s->len);
    double* rho1 = (double*)malloc(sizeof(double) * s->len);
    if (!rho0 || !rho1) { free(rho0); free(rho1); return -2; }
    for (int it = 0; it < nsteps; ++it) {
        if (s->step % s->g.sort_every == 0) {
            int r = or_sort(s);
            if (r) { free(rho0); free(rho1); return r; }
        }
        if (s->track) deposit_rho(s, rho0);
        double I[3];
        particle_step(s, I);
        if (series_push(s, I)) { free(rho0); free(rho1); return -2; }
        if (s->track) {
        deposit_rho(s, rho1);
        /* continuity of the deposited current: (rho1 - rho0)/dt + div J */
        double res = 0.0, scale = 0.0;
        for (long k = 0; k < valid_len(s, 2, 0); ++k)
            for (long j = 0; j < valid_len(s, 1, 0); ++j)
                for (long i = 0; i < valid_len(s, 0, 0); ++i) {
                    long ijk[3] = {i, j, k};
                    int interior = 1;
                    for (int a = 0; a < 3; ++a)
                        if (is_open(s, a) && (ijk[a] == 0 || ijk[a] == s->g.n[a])) interior = 0;
                    if (!interior) continue;
                    size_t q = fidx(s, i, j, k);
                    double div = dbwd(s, s->J[0], i, j, k, 0) + dbwd(s, s->J[1], i, j, k, 1) +
                                 dbwd(s, s->J[2], i, j, k, 2);
                    double r = fabs((rho1[q] - rho0[q]) / s->g.dt + div);
                    if (r > res) res = r;
                    double sc = fabs(rho1[q]) / s->g.dt;
                    if (sc > scale) scale = sc;
                }
        s->cont_res = res;
        s->cont_scale = scale;
        }
        b_half_step(s);
        e_step(s, ((double)s->step + 0.5) * s->g.dt);
        b_half_step(s);
        s->step++;
    }
    free(rho0);
    free(rho1);
    return 0;
}

double or_last_continuity_residual(const or_sim* s, double* scale)
{
    if (scale) *scale = s->cont_scale;
    return s->cont_res;
}

/* ------------------------------------------------------------------------- */
/* Fields in and out, initial fields, diagnostics                            */
/* ------------------------------------------------------------------------- */
size_t or_field_len(const or_sim* s) { return s->len; }
void or_field_shape(const or_sim* s, int L[3]) { for (int a = 0; a < 3; ++a) L[a] = s->L[a]; }

int or_get_fields(const or_sim* s, double* e, double* b)
{
    for (int c = 0; c < 3; ++c) {
        if (e) memcpy(e + c * s->len, s->E[c], sizeof(double) * s->len);
        if (b) memcpy(b + c * s->len, s->B[c], sizeof(double) * s->len);
    }
    return 0;
}

int or_set_fields(or_sim* s, const double* e, const double* b)
{
    for (int c = 0; c < 3; ++c) {
        if (e) memcpy(s->E[c], e + c * s->len, sizeof(double) * s->len);
        if (b) memcpy(s->B[c], b + c * s->len, sizeof(double) * s->len);
    }
    return 0;
}

int or_set_ext_field(or_sim* s, const double* e)
{
    if (e)
        for (size_t q = 0; q < 3 * s->len; ++q)
            if (!isfinite(e[q])) return -1;
    for (int c = 0; c < 3; ++c) {
        free(s->eext[c]);
        s->eext[c] = NULL;
        if (!e) continue;
        s->eext[c] = (double*)malloc(sizeof(double) * s->len);
        if (!s->eext[c]) return -2;
        memcpy(s->eext[c], e + c * s->len, sizeof(double) * s->len);
    }
    return 0;
}

int or_set_eps_inv(or_sim* s, const double* einv)
{
    if (einv)
        for (size_t q = 0; q < 3 * s->len; ++q)
            if (!(einv[q] > 0.0) || !isfinite(einv[q])) return -1;
    for (int c = 0; c < 3; ++c) {
        free(s->einv[c]);
        s->einv[c] = NULL;
        if (!einv) continue;
        s->einv[c] = (double*)malloc(sizeof(double) * s->len);
        if (!s->einv[c]) return -2;
        memcpy(s->einv[c], einv + c * s->len, sizeof(double) * s->len);
    }
    return 0;
}

/* Off-diagonal entries may be nonzero only where, on every open axis, the
 * node index lies in [2, n - 2]: the averaged update terms then come from
 * interior nodes (never a Mur face or padding). */
int or_set_eps_offdiag(or_sim* s, const double* e)
{
    if (e) {
        for (int m = 0; m < 6; ++m) {
            int a = m / 2;
            int half[3];
            stag_E(a, half);
            for (int k = 0; k < s->L[2]; ++k)
                for (int j = 0; j < s->L[1]; ++j)
                    for (int i = 0; i < s->L[0]; ++i) {
                        double v = e[(size_t)m * s->len + ((size_t)k * s->L[1] + j) * s->L[0] + i];
                        if (!isfinite(v)) return -1;
                        if (v == 0.0) continue;
                        int ijk[3] = {i, j, k};
                        for (int x = 0; x < 3; ++x)
                            if (is_open(s, x) && (ijk[x] < 2 || ijk[x] > s->g.n[x] - 2)) return -1;
                    }
        }
    }
    for (int m = 0; m < 6; ++m) {
        free(s->eoff[m]);
        s->eoff[m] = NULL;
        if (!e) continue;
        s->eoff[m] = (double*)malloc(sizeof(double) * s->len);
        if (!s->eoff[m]) return -2;
        memcpy(s->eoff[m], e + (size_t)m * s->len, sizeof(double) * s->len);
    }
    return 0;
}

int or_get_current(const or_sim* s, double* j)
{
    for (int c = 0; c < 3; ++c) memcpy(j + c * s->len, s->J[c], sizeof(double) * s->len);
    return 0;
}

/* Fixed ion background (Sec. 2: ions are fixed).  uniform = 1: the mean of
 * -rho_e; uniform = 0: -rho_e at t = 0 node by node. */
int or_set_ion_background(or_sim* s, int uniform)
{
    deposit_rho(s, s->rho_ion);
    size_t nn = 0;
    double sum = 0.0;
    for (long k = 0; k < valid_len(s, 2, 0); ++k)
        for (long j = 0; j < valid_len(s, 1, 0); ++j)
            for (long i = 0; i < valid_len(s, 0, 0); ++i) { sum += s->rho_ion[fidx(s, i, j, k)]; ++nn; }
    for (size_t q = 0; q < s->len; ++q)
        s->rho_ion[q] = uniform ? -sum / (double)nn : -s->rho_ion[q];
    s->have_ion = 1;
    return 0;
}

/* 1D periodic: E_x from the discrete Gauss law over rho_e + rho_ion,
 * D_x(i+1/2) = D_x(i-1/2) + dx rho_i / eps0 with D_x / eps0 = eps E_x of zero
 * mean, then E_x = einv D_x / eps0 (E_x itself for the unit tensor). */
int or_gauss_init_1d(or_sim* s)
{
    if (s->g.dims != 1 || !s->g.periodic[0] || !s->have_ion) return -1;
    long n = s->g.n[0];
    double* rho = (double*)malloc(sizeof(double) * s->len);
    if (!rho) return -2;
    deposit_rho(s, rho);
    double run = 0.0, mean = 0.0;
    for (long i = 0; i < n; ++i) {
        /* node i+1 lies between E_x(i+1/2) and E_x(i+3/2) */
        /* node i lies between E_x(i-1/2) (index i-1) and E_x(i+1/2) (index i) */
        run += s->g.dx[0] * (rho[i] + s->rho_ion[i]) / EPS0;
        s->E[0][i] = run;
    }
    for (long i = 0; i < n; ++i) mean += s->E[0][i];
    mean /= (double)n;
    for (long i = 0; i < n; ++i) {
        s->E[0][i] -= mean;
        if (s->einv[0]) s->E[0][i] *= s->einv[0][i];
    }
    free(rho);
    return 0;
}

double or_field_energy(const or_sim* s)
{
    double mu0 = 1.0 / (EPS0 * CLIGHT * CLIGHT), dv = dvol(s), u = 0.0;
    for (int c = 0; c < 3; ++c) {
        int hE[3], hB[3];
        stag_E(c, hE);
        stag_B(c, hB);
        for (long k = 0; k < valid_len(s, 2, hE[2]); ++k)
            for (long j = 0; j < valid_len(s, 1, hE[1]); ++j)
                for (long i = 0; i < valid_len(s, 0, hE[0]); ++i) {
                    /* electric energy density eps0 eps E^2 / 2 (eps = 1 / einv) */
                    size_t q = fidx(s, i, j, k);
                    double e = s->E[c][q];
                    u += 0.5 * EPS0 * e * e * dv / (s->einv[c] ? s->einv[c][q] : 1.0);
                }
        for (long k = 0; k < valid_len(s, 2, hB[2]); ++k)
            for (long j = 0; j < valid_len(s, 1, hB[1]); ++j)
                for (long i = 0; i < valid_len(s, 0, hB[0]); ++i) {
                    double b = s->B[c][fidx(s, i, j, k)];
                    u += 0.5 / mu0 * b * b * dv;
                }
    }
    return u;
}

double or_kinetic_energy(const or_sim* s, int sid)
{
    if (sid < 0 || sid >= s->nsp) return NAN;
    const sp_state* st = &s->sp[sid];
    double e = 0.0;
    for (size_t p = 0; p < st->n; ++p) {
        const double* v = &st->v[3 * p];
        e += 0.5 * st->sp.m * st->sp.weight * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    }
    return e;
}

/* max over interior nodes of |div D / eps0 - (rho_e + rho_ion) / eps0| with
 * D / eps0 = eps E (eps = 1 / einv per component; E itself for the unit tensor). */
double or_gauss_residual(const or_sim* s, double* scale)
{
    double* rho = (double*)malloc(sizeof(double) * s->len);
    double* D[3] = {NULL, NULL, NULL};
    if (!rho) return NAN;
    for (int c = 0; c < 3; ++c) {
        D[c] = (double*)malloc(sizeof(double) * s->len);
        if (!D[c]) { for (int d = 0; d < c; ++d) free(D[d]); free(rho); return NAN; }
        for (size_t q = 0; q < s->len; ++q) D[c][q] = s->einv[c] ? s->E[c][q] / s->einv[c][q] : s->E[c][q];
    }
    deposit_rho(s, rho);
    double res = 0.0, sc = 0.0;
    for (long k = 0; k < valid_len(s, 2, 0); ++k)
        for (long j = 0; j < valid_len(s, 1, 0); ++j)
            for (long i = 0; i < valid_len(s, 0, 0); ++i) {
                long ijk[3] = {i, j, k};
                int interior = 1;
                for (int a = 0; a < 3; ++a)
                    if (is_open(s, a) && (ijk[a] == 0 || ijk[a] == s->g.n[a])) interior = 0;
                if (!interior) continue;
                size_t q = fidx(s, i, j, k);
                double div = dbwd(s, D[0], i, j, k, 0) + dbwd(s, D[1], i, j, k, 1) +
                             dbwd(s, D[2], i, j, k, 2);
                double r = fabs(div - (rho[q] + (s->have_ion ? s->rho_ion[q] : 0.0)) / EPS0);
                if (r > res) res = r;
                if (fabs(rho[q]) / EPS0 > sc) sc = fabs(rho[q]) / EPS0;
            }
    for (int c = 0; c < 3; ++c) free(D[c]);
    free(rho);
    if (scale) *scale = sc;
    return res;
}

/* Sec. 2 relaxation study: histogram of the macroparticle kinetic energies
 * 0.5 m |v|^2 of species sid in nbins equal bins over [0, e_max) (joules);
 * counts[nbins] takes the energies at or above e_max.  Reading: the paper
 * histograms macroparticles (not weighted by the real-particle weight). */
int or_energy_histogram(const or_sim* s, int sid, double e_max, int nbins, uint64_t* counts)
{
    if (sid < 0 || sid >= s->nsp || nbins < 1 || !(e_max > 0.0)) return -1;
    const sp_state* st = &s->sp[sid];
    for (int b = 0; b <= nbins; ++b) counts[b] = 0;
    for (size_t p = 0; p < st->n; ++p) {
        const double* v = &st->v[3 * p];
        double e = 0.5 * st->sp.m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        double f = e / e_max * (double)nbins;
        long b = f >= (double)nbins ? nbins : (long)f;
        counts[b] += 1;
    }
    return 0;
}

int or_current_series(const or_sim* s, double* out, size_t cap, size_t* n)
{
    if (n) *n = s->series_n;
    if (!out) return 0;
    size_t m = s->series_n < cap ? s->series_n : cap;
    memcpy(out, s->series, sizeof(double) * 3 * m);
    return 0;
}

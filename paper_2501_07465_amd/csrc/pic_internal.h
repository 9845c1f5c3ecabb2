// pic_internal.h -- device-resident descriptors of libpic (internal to the library).
//
// Every kernel reads its simulation from a SimDev table in device memory rather
// than from kernel arguments, so a single simulation is a batch of one and the
// batched form reuses the same kernels (membership changes rewrite the table;
// captured graphs stay valid).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int MAXSP = 4;
constexpr int MAX_BATCH = 64;

// Physical constants (CODATA 2018; e, c, hbar, kB exact).
constexpr double kQe = 1.602176634e-19;
constexpr double kMe = 9.1093837015e-31;
constexpr double kC = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kHbar = 1.054571817e-34;
constexpr double kKb = 1.380649e-23;
constexpr double kPi = 3.14159265358979323846;

enum Kind { FREE = 0, BOUND = 1, DIRAC = 2 };
enum Region { R_ALL = 0, R_BALL = 1, R_BOX = 2 };

// Halo widths of the particle-tile windows (cells, per active axis).  A particle
// may sit up to one cell outside its tile between sorts.  Gather reads nodes
// c0-1..c0+1 of the start cell c0, so the field window spans [lo-2, hi+2].  The
// charge-conserving deposit writes nodes c0..c0+1 for a move inside its start
// cell and c0-1..c0+2 for a move that leaves it; the current window spans
// [lo-1, hi+2], which holds the in-cell moves of every particle of the window
// and the cell-leaving moves of particles that start inside the tile.  The rare
// cell-leaving moves of particles that start in the one-cell ring around the
// tile add to the global current directly; with them the deposits of a tile
// reach [lo-2, hi+3] (the reach the field kernel tests).
// Per-wavefront LDS scratch of the particle kernel (values): the global gather of a particle
// outside its tile window stages 6 components x 2^3 nodes there.
constexpr int kStrayScratch = 48;

// Field-kernel tile (cells) per number of active axes: x, y, z.
template <int DIM>
struct FieldTile;
template <>
struct FieldTile<1> { static constexpr int X = 256, Y = 1, Z = 1; };
template <>
struct FieldTile<2> { static constexpr int X = 61, Y = 5, Z = 1; };  // row-sweep task: 61 columns of a wavefront, 5 rows
// rows of a row-sweep task in a simulation with a per-cell permittivity (its kernel keeps a deeper
// load ring and is faster on taller tasks)
constexpr int kSweepRowsEps = 6;
template <>
struct FieldTile<3> { static constexpr int X = 61, Y = 3, Z = 10; };  // plane-march task: 61 columns, 3 rows, 10 planes
// XCDs of the MI355X: workgroups are dispatched to them round-robin
constexpr int kXcds = 8;
// device words of a particle-kernel unit queue: a next-unit counter and a finished-block counter
// per XCD (zero between launches)
constexpr int kUnitQueueWords = 2 * kXcds;

// rows of a plane-march task in the FP64 form (its slabs of doubles take twice the registers: with
// three rows it held one wavefront per SIMD)
constexpr int kPlaneRowsFp64 = 2;
// fewest plane-march tasks a grid is split into before its plane chunks are shortened (about two
// wavefronts per SIMD of the 256 CUs)
constexpr int kFieldTasksMin = 2048;

constexpr int kGL = 2;       // low-side halo of the field window (and low reach of a tile's deposits)
constexpr int kGHf = 2;      // high-side halo of the field window
constexpr int kGHj = 3;      // high reach of a tile's deposits
constexpr int kJL = 1;       // low-side halo of the current window
constexpr int kJH = 2;       // high-side halo of the current window

// The current is accumulated in quanta: every deposit value is rounded to a whole number of
// quanta 1 / jq and added as an integer-valued FP64 number, so each sum is exact and the same in
// any order of the additions (LDS and global atomics alike): a run, its replay and the same
// simulation in a batch give bit-identical currents.  jq = 2^kJqBits / K with K the smallest
// power of two at or above the largest single deposit value of the simulation (a charge moving a
// whole cell per step, or at the speed of light along an invariant axis), so one value is at most
// 2^kJqBits quanta and sums stay exact up to 2^(53 - kJqBits) such values per node.  The FP64 form
// also keeps the fraction of each value below one quantum, in units of 2^-kJqLoBits quanta, in a
// second word, so it adds the FP64 values exactly.
constexpr int kJqBits = 36;
constexpr int kJqLoBits = 40;
constexpr double kJqLoScale = 0x1p40;  // 2^kJqLoBits
static_assert(kJqLoScale == (double)(1ll << kJqLoBits), "fraction scale");
// The particles' charge density (Gauss-law initialisation and residual) is summed the same way,
// both words for both forms, with rhoq quanta per C/m^3 from the largest single contribution.
template <typename R>
struct JWords;
template <>
struct JWords<float> { static constexpr int n = 1; };
template <>
struct JWords<double> { static constexpr int n = 2; };

struct SpeciesDev {
    int kind, reflect, region, sheet_normal;
    int n;                 // particle count
    int sortable;          // 0 for bound species after their first sort (anchors never move)
    double qm;             // q / m
    double qw;             // q * weight
    double mw;             // m * weight
    double mass;           // m
    double q;              // charge
    int mpp;               // Dirac: per-carrier q / m_d in xi[0]
    double w2[3], gam[3];  // bound: omega_b^2, gamma_b
    double bw;             // bound: weight of the magnetic force
    double vf;             // Dirac: Fermi speed
    double rc[3], rr, rlo[3], rhi[3];  // region (cell units)
    unsigned long long seed;           // Philox key of the loader and of diffusive wall draws
    // state, structure of arrays; R = float or double by precision
    int* cell;             // packed cell index (free/Dirac: current cell; bound: anchor cell)
    void* off[3];          // in-cell offset in [0,1) (bound: anchor offset)
    void* v[3];            // velocity v_{n-1/2} [m/s]
    void* xi[3];           // bound: displacement from the anchor [m]
    // second copy for the sort permutation (pointers swapped after each sort)
    int* cell_alt;
    void* off_alt[3];
    void* v_alt[3];
    void* xi_alt[3];
    int* tile_start;       // [ntiles + 1] first particle of each tile
    // sort scratch
    int* keys;
    int* keys_alt;
    int* vals;
    int* vals_alt;
};

struct SimDev {
    int dims, precision, nspecies, ntiles;
    int n[3], L[3], periodic[3], T[3], Tshift[3], ntile[3];
    int Wf[3], Wj[3];      // particle-window extents (1 on inactive axes)
    int gl[3];             // low halo per axis (kGL on active axes, 0 otherwise)
    int Vf, Vj;            // window volumes
    int pshift[3], pmask[3];  // packed cell: c = (cell >> pshift) & pmask
    int FT[3], nft[3], nftiles;  // field tiles
    long long Lvol;
    double dx[3], inv_dx[3], dt_dx[3], dt;
    double mur_k[3];       // (c dt - dx) / (c dt + dx)
    // fields, planar [comp][z][y][x], R; two buffers: step n reads [n & 1] and writes [(n+1) & 1]
    void* E[2][3];
    void* B[2][3];
    int* tile_slot;        // [ntiles]: first unit of an active tile, -1 otherwise
    int* tile_nslot;       // [ntiles]: units of an active tile (consecutive)
    int* active;           // [ntiles]: active tile list
    int* n_active;         // device scalar
    int max_slots;         // capacity of the active list (tiles that can hold particles)
    int* units;            // [max_units][3]: tile, first and end particle in the tile's
                           // species-concatenated order
    int* n_units;          // device scalar
    int max_units;         // capacity of the unit list
    int unit_cap;          // most particles per unit (0: one unit per tile)
    int* sort_hist;        // radix-sort digit histogram scratch
    int* sort_part;        // radix-sort digit totals [8][256] (copies summed by the row scan)
    double* J[2];          // [words][3][Lvol] J^{n+1/2} by step parity, in quanta (integer-valued
                           // FP64; FP32 form one word, FP64 form two: quanta and their fraction in
                           // units of 2^-kJqLoBits): every tile's current window is added by exact
                           // atomics, deposits outside the windows add directly
    double jq, jq_inv;     // quanta per unit of current density, and its inverse (powers of two)
    int* fdirty;           // [2][nftiles] where the owned nodes of J[p] hold deposits: 1D tiles 0/1; 2D, 3D tasks a bit per particle-tile column (~0: all)
    long long* over_stamp; // [2] step+1 of the last overflow per parity
    unsigned long long* over_count;
    int* nonfinite;        // set to 1 by the particle kernel when a pushed velocity is not finite
    double* partials;      // [max_units][3] per unit: sum q w v_{n+1/2}
    double* series;        // [series_cap][3]
    int series_cap;
    long long* step_p;     // steps pushed (written by the particle kernel)
    long long* step_f;     // steps whose fields are done (written by the field kernel)
    // source
    int src_kind, src_comp, src_axis, src_index[3];
    double src_j0, src_omega, src_tau;
    // diagnostics
    int track;             // keep the merged particle current of the last step
    void* jtrack;          // [3][Lvol] R
    void* einv;            // [3][Lvol] R: inverse permittivity at the E_c nodes, or null (unit tensor)
    void* eoff;            // [6][Lvol] R: off-diagonal inverse permittivity (a, b) at the E_a nodes,
                           // order 01 02 10 12 20 21, or null (diagonal tensor)
    void* tu;              // [3][Lvol] R: update terms c^2 curl B - J / eps0 of the full-tensor step
    int* tlist;            // [2][Lvol]: nodes whose update terms are averaged, then nodes with an
                           // off-diagonal row (ascending; built when the entries are loaded)
    int* tcount;           // [2]: lengths of the two lists
    void* eext;            // [3][Lvol] R: static external field at the E_c nodes felt by the particles, or null
    double* rho_ion;       // [Lvol]
    double* rho_a;         // [Lvol]
    double* rho_b;         // [Lvol]
    double* rho_lo;        // [Lvol]: fraction words of the exact charge-density sum
    double rhoq, rhoq_inv; // quanta of charge density per C/m^3, and its inverse (powers of two)
    double* red;           // reduction scratch
    unsigned long long* hist;  // [kMaxHistBins + 1] energy-histogram counts
    SpeciesDev sp[MAXSP];
};

// ---- small host/device helpers ----------------------------------------------------------------
// Packed cell: the fields fill all 32 bits (2D: 16 + 16, 3D: 11 + 11 + 10), so packing and
// unpacking run on unsigned values; the stored int is only ever unpacked, never compared.  The
// layout depends only on the dimension: per dimension, the shift and the mask of each field.
constexpr int kCellShift[3][3] = {{0, 0, 0}, {0, 16, 0}, {0, 11, 22}};
constexpr int kCellMask[3][3] = {{0x7fffffff, 0, 0}, {0xffff, 0xffff, 0}, {0x7ff, 0x7ff, 0x3ff}};

// the same with the dimension known at compile time (shifts and masks as immediates)
template <int DIM>
__host__ __device__ inline int pack_cell_d(int i, int j, int k)
{
    constexpr int s0 = kCellShift[DIM - 1][0], s1 = kCellShift[DIM - 1][1], s2 = kCellShift[DIM - 1][2];
    return (int)(((unsigned)i << s0) | ((unsigned)j << s1) | ((unsigned)k << s2));
}
template <int DIM>
__host__ __device__ inline void unpack_cell_d(int c, int out[3])
{
    constexpr int s0 = kCellShift[DIM - 1][0], s1 = kCellShift[DIM - 1][1], s2 = kCellShift[DIM - 1][2];
    constexpr unsigned m0 = kCellMask[DIM - 1][0], m1 = kCellMask[DIM - 1][1], m2 = kCellMask[DIM - 1][2];
    const unsigned u = (unsigned)c;
    out[0] = (int)((u >> s0) & m0);
    out[1] = (int)((u >> s1) & m1);
    out[2] = (int)((u >> s2) & m2);
}

__host__ __device__ inline int pack_cell(const SimDev& S, int i, int j, int k)
{
    return (int)(((unsigned)i << S.pshift[0]) | ((unsigned)j << S.pshift[1]) | ((unsigned)k << S.pshift[2]));
}

__host__ __device__ inline void unpack_cell(const SimDev& S, int c, int out[3])
{
    const unsigned u = (unsigned)c;
    out[0] = (int)((u >> S.pshift[0]) & (unsigned)S.pmask[0]);
    out[1] = (int)((u >> S.pshift[1]) & (unsigned)S.pmask[1]);
    out[2] = (int)((u >> S.pshift[2]) & (unsigned)S.pmask[2]);
}

// Tile-major cell key: tile id, then the cell inside the tile (x fastest).
__host__ __device__ inline int cell_key(const SimDev& S, const int c[3])
{
    int tid = ((c[2] >> S.Tshift[2]) * S.ntile[1] + (c[1] >> S.Tshift[1])) * S.ntile[0] + (c[0] >> S.Tshift[0]);
    int loc = (((c[2] & (S.T[2] - 1)) << S.Tshift[1]) + (c[1] & (S.T[1] - 1))) << S.Tshift[0];
    loc += c[0] & (S.T[0] - 1);
    return (tid << (S.Tshift[0] + S.Tshift[1] + S.Tshift[2])) + loc;
}

// LDS bytes of a particle-kernel workgroup: the E, B window and the per-wavefront stray scratch
// (reals), rounded up to 8 bytes, then the current window (FP64 words).
inline size_t particle_lds_bytes(bool fp64, int vf, int vj, int block)
{
    const size_t es = fp64 ? 8 : 4;
    size_t f = es * (6 * (size_t)vf + (size_t)kStrayScratch * (size_t)(block / 64));
    f = (f + 7) / 8 * 8;
    return f + 8 * (size_t)(fp64 ? JWords<double>::n : JWords<float>::n) * 3 * (size_t)vj;
}

// ---- launchers (defined in the kernel translation units) ---------------------------------------
struct Launch {
    const SimDev* sims;    // device table
    int nsims;
    int max_vf, max_vj;    // LDS sizing over members
    int pgrid;             // particle-kernel grid
    int block;             // particle-kernel block
    int ftiles_total;      // field tiles over members
    bool eps;              // some member has a per-cell inverse permittivity
    bool rare;             // some member has a species with diffusive walls
    bool ext;              // some member has a static external field or per-carrier Dirac mass
    long long tensor_lvol; // field nodes of a simulation with a full tensor (0: none; a batch launches
                           // each tensor member's passes itself, through Launchers::tensor)
    int tile[3];           // the particle tile shape shared by every member (0 if they differ)
    unsigned* queue;       // the particle kernel's unit queue (kUnitQueueWords, zero between launches)
    int ncu;               // compute units of the device (the particle grid is fitted to them; 0: L.pgrid)
    int permask;           // the members' periodic active axes, a bit per axis (-1 if they differ)
    hipStream_t stream;
};

struct LoadArgs {
    int s, sid, ppc, ncell, momentum, loading, pert_mode, ntab;
    unsigned long long seed;
    double e_fermi, kT, mass, pert_amp, xi_radius, e_max;
    const int* cells;     // packed region cells, row-major order
    const double* cdf;    // FD CDF on x = sqrt(e / e_max), ntab + 1 nodes
};

// Launchers of the precision-templated kernels; explicitly instantiated for float (pic_k32.hip)
// and double (pic_k64.hip).
constexpr int kMaxHistBins = 4096;  // most bins of pic_energy_histogram

template <typename R>
struct Launchers {
    static hipError_t particles(int dims, const Launch& L);
    static hipError_t fields(int dims, const Launch& L, int lds_elems);
    // the full-tensor passes of one simulation (its device table entry, its field nodes)
    static hipError_t tensor(int dims, const SimDev* entry, long long lvol, hipStream_t st);
    static hipError_t load(int dims, SimDev* dS, const LoadArgs& A, hipStream_t st);
    static hipError_t field_energy(const SimDev* dS, int par, double* part, int nb, hipStream_t st);
    static hipError_t kinetic(const SimDev* dS, int s, double* part, int nb, hipStream_t st);
    static hipError_t energy_hist(const SimDev* dS, int s, double e_max, int nbins, unsigned long long* counts,
                                  hipStream_t st);
    static hipError_t rho(int dims, const SimDev* dS, double* rho, int nb, hipStream_t st);
    static hipError_t gauss(int dims, const SimDev* dS, int par, const double* rho, double* part, int nb, hipStream_t st);
    static hipError_t continuity(int dims, const SimDev* dS, double* part, int nb, hipStream_t st);
    static hipError_t gauss_init_1d(const SimDev* dS, int par, const double* rho, hipStream_t st);
};

// Untyped helpers (pic_sort.hip).
hipError_t enqueue_fill(void* p, size_t bytes, hipStream_t st);  // zero fill by kernel (graph safe)
hipError_t enqueue_fill_pattern(void* p, size_t bytes, unsigned lo, unsigned hi, hipStream_t st);  // 64-bit pattern
hipError_t enqueue_sum(const double* x, long long n, double* part, int nb, hipStream_t st);
hipError_t enqueue_final(const double* part, int nb, int nv, int op, double* out, hipStream_t st);
hipError_t enqueue_ion(SimDev* dS, const double* rho, int uniform, const double* total, hipStream_t st);

}  // namespace pic

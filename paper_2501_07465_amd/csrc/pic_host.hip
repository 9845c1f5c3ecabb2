// pic_host.hip -- host side of libpic: the C ABI of include/pic.h.
//
// Validates descriptors, plans the device arena (the library never allocates device memory),
// builds the loader tables, enqueues the loaders, the cell sort, the particle and field kernels
// and the FP64 diagnostics on the caller's stream, and optionally replays one sort period of
// steps as a HIP graph.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pic.h"
#include "pic_internal.h"
#include "pic_sort.h"

using namespace pic;

namespace {

constexpr int kFdTab = 65536;       // FD inverse-CDF intervals
constexpr int kDiagBlocks = 1024;   // blocks of the diagnostic reductions
constexpr size_t kAlign = 256;

struct SpeciesHost {
    pic_species_desc d;
    uint64_t seed = 0;
    long long n = 0;
    double density = 0.0, weight = 0.0, mass = 0.0;
    std::vector<int> cells;       // packed region cells (loader)
    std::vector<double> cdf;      // FD table (loader, T > 0)
    double e_max = 0.0;
    // device buffers: [0] and [1] copies; parity says which is current
    int* cell[2] = {nullptr, nullptr};
    void* off[2][3] = {};
    void* v[2][3] = {};
    void* xi[2][3] = {};
    int parity = 0;
    int* dcells = nullptr;
    double* dcdf = nullptr;
    bool sorted_once = false;
};

}  // namespace

struct pic_sim {
    pic_grid_desc g{};
    std::vector<SpeciesHost> sp;
    SimDev h{};              // host mirror of the device table
    SimDev* d = nullptr;     // device table (in the arena)
    char* arena = nullptr;
    size_t arena_bytes = 0;
    hipStream_t st = nullptr;
    bool bound = false;
    long long step = 0;
    bool need_sort = true;
    std::string err;
    int es = 4;              // element size of reals
    int passes = 1;
    int pgrid = 1;
    int ncu = 0;                 // compute units of the device at pic_bind
    unsigned* pqueue = nullptr;  // the particle kernel's unit queue (in the arena, zeroed at bind)
    int field_lds = 0;
    int max_slots = 0;
    bool graphs = false;
    hipGraphExec_t gexec = nullptr;
    std::vector<int> graph_species;  // species sorted inside the captured period
    double* part = nullptr;  // diagnostic partials [kDiagBlocks * 4]
    double* outv = nullptr;  // diagnostic results [16]
    double* cont = nullptr;  // last continuity residual [2]
    int batch_refs = 0;      // member of a batch
    SimDev* d_batch = nullptr;  // the member's entry in the batch table
    int bslot = -1;          // its slot
    hipGraphExec_t bsort = nullptr;  // its periodic sorts in the batch (against its entry)
    pic_batch* owner = nullptr;      // the batch it is in
    int device = 0;          // the GPU current at pic_bind (the arena's and the stream's)
    double einv_max = 1.0;   // largest loaded inverse permittivity (1 for the unit tensor)
    double eoff_max = 0.0;   // largest row sum of |off-diagonal inverse permittivity|
};

// The device table the kernels of this simulation must read: its own, or its batch entry.
static SimDev* dtab(pic_sim* s) { return s->batch_refs ? s->d_batch : s->d; }

struct pic_batch;

static int fail(pic_sim* s, int code, const char* fmt, ...)
{
    if (s) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        s->err = buf;
    }
    return code;
}

static thread_local std::string g_create_err;

static int scratch_address(pic_sim* s, int dev, unsigned long long** out);

#define HIPCHK(sim, expr)                                                                           \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(sim, PIC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

static bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
static int ilog2(int x) { int r = 0; while ((1 << r) < x) ++r; return r; }

// ---------------------------------------------------------------------------------------------
// Closed forms the loader needs (Sec. 2, Sec. 5, eq:dtlimit)
// ---------------------------------------------------------------------------------------------
// Density of a free-electron gas with Fermi energy E_F: n = (2 m E_F / hbar^2)^{3/2} / (3 pi^2)
// (the Fermi-energy relation of Sec. 2 with exponent 2/3 on (3 pi^2 n)).
static double density_from_fermi(double ef, double m)
{
    return std::pow(2.0 * m * ef / (kHbar * kHbar), 1.5) / (3.0 * kPi * kPi);
}

// Dirac sheet density with fourfold degeneracy, n_2D = (E_F / (hbar v_F))^2 / pi.
static double dirac_density2d(double ef, double vf)
{
    const double kf = ef / (kHbar * vf);
    return kf * kf / kPi;
}

// m_d = p_F / (2 v_F), p_F = E_F / v_F (Sec. 5)
static double dirac_mass(double ef, double vf) { return (ef / vf) / (2.0 * vf); }

// ---------------------------------------------------------------------------------------------
// Grid validation and derived geometry
// ---------------------------------------------------------------------------------------------
static int setup_grid(pic_sim* s)
{
    pic_grid_desc& g = s->g;
    SimDev& h = s->h;
    if (g.dims < 1 || g.dims > 3) return fail(s, PIC_EINVAL, "dims must be 1, 2 or 3");
    if (!(g.dt > 0.0) || !std::isfinite(g.dt)) return fail(s, PIC_EINVAL, "dt must be positive");
    if (g.precision != PIC_FP32 && g.precision != PIC_FP64) return fail(s, PIC_EINVAL, "precision");
    if (g.sort_every < 1) g.sort_every = 20;
    if (g.block == 0) g.block = 256;
    if (g.block != 64 && g.block != 128 && g.block != 256 && g.block != 512)
        return fail(s, PIC_EINVAL, "block must be 64, 128, 256 or 512");
    if (g.series_cap <= 0) g.series_cap = 8192;
    if (g.unit < 0 || (g.unit > 0 && g.unit < 64)) return fail(s, PIC_EINVAL, "unit must be 0 or >= 64");
    if (g.eps_cells < 0 || g.eps_cells > 2) return fail(s, PIC_EINVAL, "eps_cells must be 0, 1 or 2");
    if (g.eps_cells == 2 && g.track_continuity)
        return fail(s, PIC_EINVAL, "a full dielectric tensor folds its off-diagonal term into the current: no continuity tracking");
    if (g.ext_field != 0 && g.ext_field != 1) return fail(s, PIC_EINVAL, "ext_field must be 0 or 1");
    memset(&h, 0, sizeof(h));
    h.unit_cap = g.unit;
    h.dims = g.dims;
    h.precision = g.precision;
    s->es = g.precision == PIC_FP32 ? 4 : 8;
    const int lim[3][3] = {{1 << 30, 1, 1}, {65535, 65535, 1}, {2047, 2047, 1023}};
    for (int a = 0; a < 3; ++a) {
        const bool act = a < g.dims;
        if (!act) {
            g.n[a] = 1;
            g.tile[a] = 1;
            g.bc[a] = PIC_PERIODIC;
            if (!(g.dx[a] > 0.0)) g.dx[a] = 1.0;
        }
        if (g.n[a] < 1 || g.n[a] > lim[g.dims - 1][a]) return fail(s, PIC_EINVAL, "n[%d] out of range", a);
        if (act && !(g.dx[a] > 0.0)) return fail(s, PIC_EINVAL, "dx[%d] must be positive", a);
        if (g.bc[a] != PIC_PERIODIC && g.bc[a] != PIC_OPEN) return fail(s, PIC_EINVAL, "bc[%d]", a);
        if (!pow2(g.tile[a])) return fail(s, PIC_EINVAL, "tile[%d] must be a power of two", a);
        if (act && g.bc[a] == PIC_OPEN && g.n[a] < 4) return fail(s, PIC_EINVAL, "open axis %d needs >= 4 cells", a);
        h.n[a] = g.n[a];
        h.periodic[a] = g.bc[a] == PIC_PERIODIC ? 1 : 0;
        h.L[a] = (act && !h.periodic[a]) ? g.n[a] + 1 : g.n[a];
        h.T[a] = g.tile[a];
        h.Tshift[a] = ilog2(g.tile[a]);
        h.ntile[a] = (g.n[a] + g.tile[a] - 1) / g.tile[a];
        if (act && h.periodic[a]) {
            const long long lo_max = (long long)(h.ntile[a] - 1) * h.T[a];
            if (2LL * g.n[a] <= lo_max + h.T[a] + 2)
                return fail(s, PIC_EINVAL, "periodic axis %d too short for tile %d", a, h.T[a]);
        }
        h.Wf[a] = act ? h.T[a] + kGL + kGHf : 1;
        h.Wj[a] = act ? h.T[a] + kJL + kJH : 1;
        h.gl[a] = act ? kGL : 0;
        h.dx[a] = g.dx[a];
        h.inv_dx[a] = 1.0 / g.dx[a];
        h.dt_dx[a] = g.dt / g.dx[a];
        h.mur_k[a] = (kC * g.dt - g.dx[a]) / (kC * g.dt + g.dx[a]);
    }
    // packed cell layout
    for (int a = 0; a < 3; ++a) {
        h.pshift[a] = kCellShift[g.dims - 1][a];
        h.pmask[a] = kCellMask[g.dims - 1][a];
    }
    long long tiles = 1;
    for (int a = 0; a < 3; ++a) tiles *= h.ntile[a];
    const long long keyspace = tiles * h.T[0] * h.T[1] * h.T[2];
    if (keyspace >= (1LL << 31)) return fail(s, PIC_EINVAL, "cell key space exceeds int32");
    h.ntiles = (int)tiles;
    int bits = 1;
    while ((1LL << bits) < keyspace) ++bits;
    s->passes = (bits + 7) / 8;
    h.Vf = h.Wf[0] * h.Wf[1] * h.Wf[2];
    h.Vj = h.Wj[0] * h.Wj[1] * h.Wj[2];
    const size_t plds = particle_lds_bytes(g.precision == PIC_FP64, h.Vf, h.Vj, g.block);
    if (plds > 65536) return fail(s, PIC_EINVAL, "particle tile needs %zu bytes of LDS (> 64 KiB)", plds);
    // field tiles
    const int ft[3][3] = {{FieldTile<1>::X, FieldTile<1>::Y, FieldTile<1>::Z},
                          {FieldTile<2>::X, FieldTile<2>::Y, FieldTile<2>::Z},
                          {FieldTile<3>::X, FieldTile<3>::Y, FieldTile<3>::Z}};
    h.Lvol = 1;
    h.nftiles = 1;
    for (int a = 0; a < 3; ++a) {
        h.FT[a] = a < g.dims ? ft[g.dims - 1][a] : 1;
        if (g.dims == 2 && a == 1 && g.eps_cells) h.FT[a] = kSweepRowsEps;
        if (g.dims == 3 && a == 1 && g.precision == PIC_FP64) h.FT[a] = kPlaneRowsFp64;
        // the 3D plane march takes row groups over all L_y rows (the last group shifted down to end
        // at the last row), columns and plane chunks over the cells (the last one also owns node n).
        // On a small grid the plane chunks are shortened until there are enough tasks to keep
        // several wavefronts per SIMD (each task's march is a chain of dependent plane loads), down
        // to two planes (one on grids of fewer than 32768 cells).
        if (g.dims == 3 && a == 2)
            while (h.FT[2] > ((long long)g.n[0] * g.n[1] * g.n[2] < 32768 ? 1 : 2) && (long long)h.nft[0] * h.nft[1] * ((g.n[2] + h.FT[2] - 1) / h.FT[2]) < kFieldTasksMin)
                h.FT[2] /= 2;
        const int span = (g.dims == 3 && a == 1) ? h.L[a] : g.n[a];
        h.nft[a] = (span + h.FT[a] - 1) / h.FT[a];
        h.nftiles *= h.nft[a];
        h.Lvol *= h.L[a];
    }
    // the full tensor's node lists hold int32 node indices
    if (g.eps_cells == 2 && h.Lvol > 0x7fffffffLL)
        return fail(s, PIC_EINVAL, "a full dielectric tensor needs fewer than 2^31 field nodes");
    int fl = 1;
    {
        int ve = 1, vb = 1, vj = 1;
        for (int a = 0; a < g.dims; ++a) { ve *= h.FT[a] + 3; vb *= h.FT[a] + 2; vj *= h.FT[a] + 1; }
        fl = g.dims == 1 ? 3 * (ve + vb + vj) : 0;  // E_n, B, J (E_{n+1} overwrites J); the 2D and 3D sweeps use none
    }
    s->field_lds = fl;
    h.dt = g.dt;
    h.series_cap = g.series_cap;
    h.track = g.track_continuity ? 1 : 0;
    h.src_kind = g.src_kind;
    h.src_comp = g.src_comp;
    h.src_axis = g.src_axis;
    for (int a = 0; a < 3; ++a) h.src_index[a] = g.src_index[a];
    h.src_j0 = g.src_j0;
    h.src_omega = g.src_omega;
    h.src_tau = g.src_tau;
    if (g.src_kind != PIC_SRC_NONE) {
        if (g.src_kind != PIC_SRC_SHEET && g.src_kind != PIC_SRC_POINT) return fail(s, PIC_EINVAL, "src_kind");
        if (g.src_comp < 0 || g.src_comp > 2 || !(g.src_tau > 0.0)) return fail(s, PIC_EINVAL, "source");
        if (g.src_kind == PIC_SRC_SHEET && (g.src_axis < 0 || g.src_axis >= g.dims)) return fail(s, PIC_EINVAL, "src_axis");
        for (int a = 0; a < g.dims; ++a)
            if ((g.src_kind == PIC_SRC_POINT || a == g.src_axis) && (g.src_index[a] < 0 || g.src_index[a] >= h.L[a]))
                return fail(s, PIC_EINVAL, "source index out of the grid");
    }
    return PIC_OK;
}

// region membership of a cell: ball: all corners inside; box: cell inside (cell units)
static bool cell_in_region(const pic_sim* s, const pic_species_desc& d, const int c[3])
{
    const int dims = s->g.dims;
    if (d.region == PIC_REGION_ALL) return true;
    if (d.region == PIC_REGION_BOX) {
        for (int a = 0; a < dims; ++a)
            if ((double)c[a] < d.rlo[a] || (double)(c[a] + 1) > d.rhi[a]) return false;
        return true;
    }
    for (int corner = 0; corner < (1 << dims); ++corner) {
        double r2 = 0.0;
        for (int a = 0; a < dims; ++a) {
            const double p = (double)(c[a] + ((corner >> a) & 1)) - d.rc[a];
            r2 += p * p;
        }
        if (r2 > d.rr * d.rr) return false;
    }
    return true;
}

extern "C" int pic_create(const pic_grid_desc* g, pic_sim** out)
{
    if (!g || !out) { g_create_err = "null argument"; return PIC_EINVAL; }
    *out = nullptr;
    pic_sim* s = new (std::nothrow) pic_sim();
    if (!s) { g_create_err = "out of host memory"; return PIC_ENOMEM; }
    s->g = *g;
    const int r = setup_grid(s);
    if (r) {
        g_create_err = s->err;
        delete s;
        return r;
    }
    g_create_err.clear();
    *out = s;
    return PIC_OK;
}

// plasma frequency squared of a species and its resonance, for eq:dtlimit
static void species_freqs(const SpeciesHost& x, double& wp2, double& wb2)
{
    wp2 = x.density * x.d.q * x.d.q / (kEps0 * x.mass);
    wb2 = 0.0;
    if (x.d.kind == PIC_BOUND)
        for (int a = 0; a < 3; ++a) wb2 = std::max(wb2, x.d.omega0[a] * x.d.omega0[a]);
}

// eq:dtlimit with all declared species (plasma frequencies add, largest resonance) and, if given,
// one more.  A dielectric scales the curl and current terms of the E update by einv, so the light
// speed squared and the plasma frequencies squared take the factor max(1, largest einv).
static int check_dt(pic_sim* s, const SpeciesHost* extra, double einv_max)
{
    double wp2 = 0.0, wb2 = 0.0;
    std::vector<const SpeciesHost*> all;
    for (auto& y : s->sp) all.push_back(&y);
    if (extra) all.push_back(extra);
    for (auto* y : all) {
        double a, b;
        species_freqs(*y, a, b);
        wp2 += a;
        wb2 = std::max(wb2, b);
    }
    const double m = std::max(1.0, einv_max);
    double cs = 0.0;
    for (int a = 0; a < s->g.dims; ++a) cs += 1.0 / (s->g.dx[a] * s->g.dx[a]);
    const double lim = 1.0 / std::sqrt(0.25 * wb2 + 0.25 * m * wp2 + m * kC * kC * cs);
    if (!(s->g.dt < lim)) return fail(s, PIC_ECFL, "dt %.6e is not below the stability limit %.6e", s->g.dt, lim);
    return PIC_OK;
}

extern "C" int pic_init_species(pic_sim* s, const pic_species_desc* d, uint64_t seed, int* species_id)
{
    if (!s || !d) return PIC_EINVAL;
    if (s->bound) return fail(s, PIC_ESTATE, "species must be declared before pic_bind");
    if ((int)s->sp.size() >= PIC_MAX_SPECIES) return fail(s, PIC_EINVAL, "too many species");
    const int dims = s->g.dims;
    SpeciesHost x;
    x.d = *d;
    x.seed = seed;
    if (d->kind < PIC_FREE || d->kind > PIC_DIRAC) return fail(s, PIC_EINVAL, "species kind");
    if (!(d->q != 0.0) || !std::isfinite(d->q)) return fail(s, PIC_EINVAL, "charge");
    if (d->region < PIC_REGION_ALL || d->region > PIC_REGION_BOX) return fail(s, PIC_EINVAL, "region");
    if (d->reflect < 0 || d->reflect > 2) return fail(s, PIC_EINVAL, "reflect must be 0, 1 or 2");
    if (d->reflect == 2 && !(d->kind == PIC_FREE || (d->kind == PIC_DIRAC && d->sheet_normal >= 0)))
        return fail(s, PIC_EINVAL, "diffusive walls are for free species and Dirac sheets");
    if (d->mass_per_particle != 0 && d->mass_per_particle != 1) return fail(s, PIC_EINVAL, "mass_per_particle must be 0 or 1");
    if (d->mass_per_particle && d->kind != PIC_DIRAC) return fail(s, PIC_EINVAL, "per-particle mass is for Dirac species");
    if (d->region == PIC_REGION_BALL)
        for (int a = 1; a < dims; ++a)
            if (s->g.dx[a] != s->g.dx[0]) return fail(s, PIC_EINVAL, "ball regions need equal cell sizes");
    x.mass = d->m;
    if (d->kind == PIC_DIRAC) {
        if (!(d->v_f > 0.0)) return fail(s, PIC_EINVAL, "Dirac species needs v_f");
        if (d->sheet_normal < -1 || d->sheet_normal > 2) return fail(s, PIC_EINVAL, "sheet_normal");
        if (x.mass == 0.0) {
            if (!(d->e_fermi > 0.0)) return fail(s, PIC_EINVAL, "Dirac mass needs e_fermi");
            x.mass = dirac_mass(d->e_fermi, d->v_f);
        }
    }
    if (!(x.mass > 0.0)) return fail(s, PIC_EINVAL, "mass must be positive");
    if (d->momentum != PIC_MOM_COLD && d->momentum != PIC_MOM_FD) return fail(s, PIC_EINVAL, "momentum");
    if (d->momentum == PIC_MOM_FD && d->kind == PIC_FREE && !(d->e_fermi > 0.0))
        return fail(s, PIC_EINVAL, "FD momenta need e_fermi");
    // particles stay inside: open axes need reflection into a region away from the faces, or a
    // bound species, or the Dirac sheet normal
    for (int a = 0; a < dims; ++a) {
        if (s->g.bc[a] != PIC_OPEN) continue;
        const bool pinned = d->kind == PIC_BOUND || (d->kind == PIC_DIRAC && d->sheet_normal == a);
        if (!pinned && !(d->reflect && d->region != PIC_REGION_ALL))
            return fail(s, PIC_EINVAL, "species %d can reach the open faces of axis %d", (int)s->sp.size(), a);
        double lo, hi;
        if (d->region == PIC_REGION_BALL) { lo = d->rc[a] - d->rr; hi = d->rc[a] + d->rr; }
        else if (d->region == PIC_REGION_BOX) { lo = d->rlo[a]; hi = d->rhi[a]; }
        else { lo = 0.0; hi = s->g.n[a]; }
        if (lo < 3.0 || hi > s->g.n[a] - 3.0) return fail(s, PIC_EINVAL, "region within 3 cells of an open face");
    }
    if (d->count > 0) {
        if (d->count >= (1LL << 31)) return fail(s, PIC_EINVAL, "count");
        x.n = d->count;
        x.weight = d->weight;
        x.density = d->density;
    } else {
        if (d->ppc < 1) return fail(s, PIC_EINVAL, "ppc");
        if (d->loading == PIC_LOAD_QUIET && dims != 1) return fail(s, PIC_EINVAL, "quiet start is 1D only");
        int c[3];
        for (c[2] = 0; c[2] < s->g.n[2]; ++c[2])
            for (c[1] = 0; c[1] < s->g.n[1]; ++c[1])
                for (c[0] = 0; c[0] < s->g.n[0]; ++c[0])
                    if (cell_in_region(s, *d, c)) x.cells.push_back(pack_cell(s->h, c[0], c[1], c[2]));
        x.n = (long long)x.cells.size() * d->ppc;
        if (x.n >= (1LL << 31)) return fail(s, PIC_EINVAL, "too many particles");
        double dens = d->density;
        if (!(dens > 0.0)) {
            if (!(d->e_fermi > 0.0)) return fail(s, PIC_EINVAL, "density or e_fermi required");
            if (d->kind == PIC_DIRAC) dens = dirac_density2d(d->e_fermi, d->v_f) / s->g.dx[d->sheet_normal >= 0 ? d->sheet_normal : 0];
            else dens = density_from_fermi(d->e_fermi, x.mass);
        }
        x.density = dens;
        double dv = 1.0;
        for (int a = 0; a < dims; ++a) dv *= s->g.dx[a];
        x.weight = dens * dv / d->ppc;
        const bool dmpp = d->kind == PIC_DIRAC && d->mass_per_particle;
        if (((d->kind == PIC_FREE && d->momentum == PIC_MOM_FD) || dmpp) && d->temperature > 0.0) {
            // inverse-CDF table of eq:fddist on x = sqrt(e/e_max), e_max = mu + 40 kT; the density of
            // states is sqrt(e) for free carriers (weight x^2) and e for Dirac carriers (x^3)
            const double mu = d->e_fermi, kT = kKb * d->temperature;
            x.e_max = mu + 40.0 * kT;
            x.cdf.resize(kFdTab + 1);
            double prev = 0.0;
            x.cdf[0] = 0.0;
            for (int k = 1; k <= kFdTab; ++k) {
                const double xx = (double)k / (double)kFdTab;
                const double e = x.e_max * xx * xx;
                const double p = (dmpp ? xx * xx * xx : xx * xx) / (1.0 + std::exp((e - mu) / kT));
                x.cdf[k] = x.cdf[k - 1] + 0.5 * (prev + p) * (1.0 / (double)kFdTab);
                prev = p;
            }
            const double tot = x.cdf[kFdTab];
            for (auto& v : x.cdf) v /= tot;
        }
    }
    if (int r = check_dt(s, &x, s->einv_max + s->eoff_max)) return r;
    const int sid = (int)s->sp.size();
    s->sp.push_back(std::move(x));
    if (species_id) *species_id = sid;
    return PIC_OK;
}

// tiles that can ever hold particles of any species (sizes the slot array)
static int count_slot_tiles(const pic_sim* s)
{
    const SimDev& h = s->h;
    std::vector<char> mark(h.ntiles, 0);
    const int dims = s->g.dims;
    for (const auto& x : s->sp) {
        double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
        bool all = false;
        const auto& d = x.d;
        for (int a = 0; a < dims; ++a) {
            if (d.region == PIC_REGION_ALL) { all = true; break; }
            double l, u;
            if (d.region == PIC_REGION_BALL) { l = d.rc[a] - d.rr; u = d.rc[a] + d.rr; }
            else { l = d.rlo[a]; u = d.rhi[a]; }
            const bool pinned = d.kind == PIC_BOUND || (d.kind == PIC_DIRAC && d.sheet_normal == a);
            if (!pinned && !d.reflect) { l = 0; u = s->g.n[a]; }
            lo[a] = l - 2.0;
            hi[a] = u + 2.0;
        }
        if (all || d.count > 0) {
            std::fill(mark.begin(), mark.end(), 1);
            continue;
        }
        int t0[3] = {0, 0, 0}, t1[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
            if (a >= dims) continue;
            t0[a] = (int)std::floor(lo[a] / h.T[a]);
            t1[a] = (int)std::floor(hi[a] / h.T[a]);
        }
        for (int z = t0[2]; z <= t1[2]; ++z)
            for (int y = t0[1]; y <= t1[1]; ++y)
                for (int xx = t0[0]; xx <= t1[0]; ++xx) {
                    int t[3] = {xx, y, z};
                    for (int a = 0; a < dims; ++a) t[a] = ((t[a] % h.ntile[a]) + h.ntile[a]) % h.ntile[a];
                    mark[(t[2] * h.ntile[1] + t[1]) * h.ntile[0] + t[0]] = 1;
                }
    }
    int n = 0;
    for (char m : mark) n += m;
    return std::max(n, 1);
}

// Bump allocator over the arena: assign == false only measures.
struct Planner {
    char* base;
    size_t off = 0;
    bool assign;
    template <typename T>
    T* take(size_t count)
    {
        off = (off + kAlign - 1) / kAlign * kAlign;
        T* p = assign ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * (count ? count : 1);
        return p;
    }
    void* takeb(size_t bytes)
    {
        off = (off + kAlign - 1) / kAlign * kAlign;
        void* p = assign ? base + off : nullptr;
        off += bytes ? bytes : 1;
        return p;
    }
};

static size_t plan(pic_sim* s, char* base, bool assign)
{
    SimDev& h = s->h;
    Planner P{base, 0, assign};
    const size_t es = s->es;
    const size_t L = (size_t)h.Lvol;
    s->d = P.take<SimDev>(1);
    for (int k = 0; k < 2; ++k) {
        for (int c = 0; c < 3; ++c) h.E[k][c] = P.takeb(L * es);
        for (int c = 0; c < 3; ++c) h.B[k][c] = P.takeb(L * es);
    }
    const size_t jw = s->g.precision == PIC_FP64 ? JWords<double>::n : JWords<float>::n;
    for (int p = 0; p < 2; ++p) h.J[p] = P.take<double>(jw * 3 * L);
    h.fdirty = P.take<int>(2 * (size_t)h.nftiles);
    s->max_slots = count_slot_tiles(s);
    h.max_slots = s->max_slots;
    // units of a tile: ceil(c_t / U) <= c_t / U + 1, so all units <= ceil(N / U) + active tiles
    long long max_units = s->max_slots;
    if (h.unit_cap > 0) {
        long long ntot = 0;
        for (auto& x : s->sp) ntot += x.n;
        max_units += (ntot + h.unit_cap - 1) / h.unit_cap;
    }
    h.max_units = (int)std::min<long long>(max_units, 1LL << 30);
    h.tile_slot = P.take<int>(h.ntiles);
    h.tile_nslot = P.take<int>(h.ntiles);
    h.active = P.take<int>(h.ntiles);
    h.n_active = P.take<int>(1);
    h.units = P.take<int>((size_t)h.max_units * 3);
    h.n_units = P.take<int>(1);
    h.step_p = P.take<long long>(1);
    h.step_f = P.take<long long>(1);
    h.over_stamp = P.take<long long>(2);
    h.over_count = P.take<unsigned long long>(1);
    h.nonfinite = P.take<int>(1);
    h.partials = P.take<double>((size_t)h.max_units * 3);
    h.series = P.take<double>((size_t)h.series_cap * 3);
    h.rho_ion = P.take<double>(L);
    h.rho_a = P.take<double>(L);
    h.rho_b = P.take<double>(L);
    h.rho_lo = P.take<double>(L);
    h.jtrack = h.track ? P.takeb(3 * L * es) : nullptr;
    h.einv = s->g.eps_cells ? P.takeb(3 * L * es) : nullptr;
    h.eoff = s->g.eps_cells == 2 ? P.takeb(6 * L * es) : nullptr;
    h.tu = s->g.eps_cells == 2 ? P.takeb(3 * L * es) : nullptr;
    h.tlist = s->g.eps_cells == 2 ? P.take<int>(2 * L) : nullptr;
    h.tcount = s->g.eps_cells == 2 ? P.take<int>(2) : nullptr;
    h.eext = s->g.ext_field ? P.takeb(3 * L * es) : nullptr;
    h.red = P.take<double>(16);
    s->pqueue = P.take<unsigned>(kUnitQueueWords);
    h.hist = P.take<unsigned long long>(kMaxHistBins + 1);
    s->part = P.take<double>(kDiagBlocks * 4);
    s->outv = P.take<double>(16);
    s->cont = P.take<double>(2);
    long long nb = 1;
    for (auto& x : s->sp) nb = std::max(nb, (x.n + sort_ipb(x.n) - 1) / sort_ipb(x.n));
    h.sort_hist = P.take<int>((size_t)256 * nb);
    h.sort_part = P.take<int>(8 * 256);
    h.nspecies = (int)s->sp.size();
    for (size_t i = 0; i < s->sp.size(); ++i) {
        SpeciesHost& x = s->sp[i];
        SpeciesDev& d = h.sp[i];
        const size_t n = (size_t)x.n;
        const bool bound = x.d.kind == PIC_BOUND;
        for (int k = 0; k < 2; ++k) {
            x.cell[k] = P.take<int>(n);
            for (int a = 0; a < 3; ++a) {
                x.off[k][a] = a < s->g.dims ? P.takeb(n * es) : nullptr;
                x.v[k][a] = P.takeb(n * es);
                // bound: displacements; Dirac with per-carrier mass: q / m_d in xi[0]
                const bool dm = x.d.kind == PIC_DIRAC && x.d.mass_per_particle && a == 0;
                x.xi[k][a] = (bound || dm) ? P.takeb(n * es) : nullptr;
            }
        }
        d.keys = P.take<int>(n);
        d.keys_alt = P.take<int>(n);
        d.vals = P.take<int>(n);
        d.vals_alt = P.take<int>(n);
        d.tile_start = P.take<int>((size_t)h.ntiles + 1);
        x.dcells = x.cells.empty() ? nullptr : P.take<int>(x.cells.size());
        x.dcdf = x.cdf.empty() ? nullptr : P.take<double>(x.cdf.size());
    }
    return P.off + kAlign;
}

// Fill the host mirror of species i from the host state (current parity).
static void mirror_species(pic_sim* s, int i)
{
    SpeciesHost& x = s->sp[i];
    SpeciesDev& d = s->h.sp[i];
    const auto& D = x.d;
    d.kind = D.kind;
    d.reflect = D.reflect;
    d.seed = x.seed;
    d.region = D.region;
    d.sheet_normal = D.kind == PIC_DIRAC ? D.sheet_normal : -1;
    d.n = (int)x.n;
    d.sortable = 1;
    d.qm = D.q / x.mass;
    d.qw = D.q * x.weight;
    d.mw = x.mass * x.weight;
    d.mass = x.mass;
    d.q = D.q;
    d.mpp = (D.kind == PIC_DIRAC && D.mass_per_particle) ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        d.w2[a] = D.kind == PIC_BOUND ? D.omega0[a] * D.omega0[a] : 0.0;
        d.gam[a] = D.kind == PIC_BOUND ? D.gamma[a] : 0.0;
        d.rc[a] = D.rc[a];
        d.rlo[a] = D.rlo[a];
        d.rhi[a] = D.rhi[a];
    }
    d.rr = D.rr;
    d.bw = D.kind == PIC_BOUND ? D.b_weight : 0.0;
    d.vf = D.v_f;
    const int p = x.parity, q = 1 - p;
    d.cell = x.cell[p];
    d.cell_alt = x.cell[q];
    for (int a = 0; a < 3; ++a) {
        d.off[a] = x.off[p][a];
        d.off_alt[a] = x.off[q][a];
        d.v[a] = x.v[p][a];
        d.v_alt[a] = x.v[q][a];
        d.xi[a] = x.xi[p][a];
        d.xi_alt[a] = x.xi[q][a];
    }
}

// Quantum of the current (see kJqBits): K is the smallest power of two at or above the largest
// single deposit value of any species, |q| w / (dt x the transverse cell area) for a move of a whole
// cell along an active axis, or |q| w c / (the cell area of the active axes) for the speed of light
// along an invariant axis (1D: y, z; 2D: z).
static void set_current_quantum(pic_sim* s)
{
    const pic_grid_desc& g = s->g;
    double kmax = 0.0;
    for (const auto& x : s->sp) {
        const double qw = std::fabs(x.d.q * x.weight);
        double area = 1.0;
        for (int a = 0; a < g.dims; ++a) area *= g.dx[a];
        for (int a = 0; a < 3; ++a) {
            const double k = a < g.dims ? qw / (g.dt * area / g.dx[a]) : qw * kC / area;
            kmax = std::max(kmax, k);
        }
    }
    int e = 0;
    if (kmax > 0.0 && std::isfinite(kmax)) e = (int)std::ceil(std::log2(kmax));
    s->h.jq = std::ldexp(1.0, kJqBits - e);
    s->h.jq_inv = std::ldexp(1.0, e - kJqBits);
    // charge density: the largest single contribution is |q| w / (cell volume of the active axes)
    double rmax = 0.0, vol = 1.0;
    for (int a = 0; a < g.dims; ++a) vol *= g.dx[a];
    for (const auto& x : s->sp) rmax = std::max(rmax, std::fabs(x.d.q * x.weight) / vol);
    int er = 0;
    if (rmax > 0.0 && std::isfinite(rmax)) er = (int)std::ceil(std::log2(rmax));
    s->h.rhoq = std::ldexp(1.0, kJqBits - er);
    s->h.rhoq_inv = std::ldexp(1.0, er - kJqBits);
}

static int upload_table(pic_sim* s)
{
    for (size_t i = 0; i < s->sp.size(); ++i) mirror_species(s, (int)i);
    HIPCHK(s, hipMemcpyAsync(s->d, &s->h, sizeof(SimDev), hipMemcpyHostToDevice, s->st));
    return PIC_OK;
}

extern "C" int pic_footprint(const pic_sim* s, size_t* bytes)
{
    if (!s || !bytes) return PIC_EINVAL;
    pic_sim tmp = *s;  // plan on a copy: measuring assigns nothing
    tmp.gexec = nullptr;
    *bytes = plan(&tmp, nullptr, false);
    return PIC_OK;
}

static hipError_t launch_load(pic_sim* s, int i)
{
    SpeciesHost& x = s->sp[i];
    LoadArgs A{};
    A.s = i;
    A.sid = i;
    A.ppc = x.d.ppc;
    A.ncell = (int)x.cells.size();
    A.momentum = x.d.momentum;
    A.loading = x.d.loading;
    A.pert_mode = x.d.pert_mode;
    A.ntab = kFdTab;
    A.seed = x.seed;
    A.e_fermi = x.d.e_fermi;
    A.kT = ((x.d.kind == PIC_FREE && x.d.momentum == PIC_MOM_FD) || (x.d.kind == PIC_DIRAC && x.d.mass_per_particle))
               ? kKb * x.d.temperature : 0.0;
    A.mass = x.mass;
    A.pert_amp = x.d.pert_amp;
    A.xi_radius = x.d.xi_radius;
    A.e_max = x.e_max;
    A.cells = x.dcells;
    A.cdf = x.dcdf;
    if (s->g.precision == PIC_FP32) return Launchers<float>::load(s->g.dims, s->d, A, s->st);
    return Launchers<double>::load(s->g.dims, s->d, A, s->st);
}

extern "C" int pic_bind(pic_sim* s, void* dev_arena, size_t bytes, void* hip_stream)
{
    if (!s) return PIC_EINVAL;
    if (s->bound) return fail(s, PIC_ESTATE, "already bound");
    if (!dev_arena) return fail(s, PIC_EINVAL, "null arena");
    if (reinterpret_cast<uintptr_t>(dev_arena) % kAlign) return fail(s, PIC_EINVAL, "arena must be 256-byte aligned");
    size_t need = 0;
    pic_footprint(s, &need);
    if (bytes < need) return fail(s, PIC_ENOMEM, "arena of %zu bytes is smaller than the footprint %zu", bytes, need);
    s->arena = reinterpret_cast<char*>(dev_arena);
    s->arena_bytes = bytes;
    s->st = reinterpret_cast<hipStream_t>(hip_stream);
    plan(s, s->arena, true);
    int dev = 0, ncu = 256;
    HIPCHK(s, hipGetDevice(&dev));
    s->device = dev;
    {
        // the static histogram scratch of this GPU (looked up once per device, with it current)
        unsigned long long* scr = nullptr;
        if (int r = scratch_address(s, dev, &scr)) return r;
    }
    {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
    }
    // the largest particle grid: a multiple of 8 (the XCD count) up to 8 workgroups per CU; each launch
    // fits it to the blocks its kernel can hold on the device at once
    s->pgrid = std::max(8, (std::min(s->h.max_units, ncu * 8) + 7) / 8 * 8);
    s->ncu = ncu;
    HIPCHK(s, enqueue_fill(s->arena, need - kAlign, s->st));
    if (s->h.einv) {
        // the unit tensor until pic_load_eps_inv: 1.0f, or 1.0 as the words (0, 0x3ff00000)
        const size_t nb = 3 * (size_t)s->h.Lvol * s->es;
        if (s->es == 4) HIPCHK(s, enqueue_fill_pattern(s->h.einv, nb, 0x3f800000u, 0x3f800000u, s->st));
        else HIPCHK(s, enqueue_fill_pattern(s->h.einv, nb, 0u, 0x3ff00000u, s->st));
    }
    s->einv_max = 1.0;
    s->eoff_max = 0.0;
    set_current_quantum(s);
    int r = upload_table(s);
    if (r) return r;
    for (size_t i = 0; i < s->sp.size(); ++i) {
        SpeciesHost& x = s->sp[i];
        if (x.d.count > 0 || x.n == 0) continue;
        HIPCHK(s, hipMemcpyAsync(x.dcells, x.cells.data(), x.cells.size() * sizeof(int), hipMemcpyHostToDevice, s->st));
        if (x.dcdf)
            HIPCHK(s, hipMemcpyAsync(x.dcdf, x.cdf.data(), x.cdf.size() * sizeof(double), hipMemcpyHostToDevice, s->st));
        HIPCHK(s, launch_load(s, (int)i));
    }
    HIPCHK(s, hipStreamSynchronize(s->st));
    s->bound = true;
    s->need_sort = true;
    s->step = 0;
    return PIC_OK;
}

extern "C" int pic_field_shape(const pic_sim* s, int L[3])
{
    if (!s || !L) return PIC_EINVAL;
    for (int a = 0; a < 3; ++a) L[a] = s->h.L[a];
    return PIC_OK;
}

extern "C" long long pic_species_count(const pic_sim* s, int sid)
{
    if (!s || sid < 0 || sid >= (int)s->sp.size()) return -1;
    return s->sp[sid].n;
}

template <typename R>
static void to_real(const double* src, size_t n, std::vector<char>& buf)
{
    buf.resize(n * sizeof(R));
    R* d = reinterpret_cast<R*>(buf.data());
    for (size_t i = 0; i < n; ++i) d[i] = R(src[i]);
}

extern "C" int pic_load_particles(pic_sim* s, int sid, const double* x, const double* v, const double* xi, size_t n)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind before loading particles");
    if (s->batch_refs) return fail(s, PIC_ESTATE, "simulation is in a batch");
    if (sid < 0 || sid >= (int)s->sp.size()) return fail(s, PIC_EINVAL, "species id");
    SpeciesHost& sp = s->sp[sid];
    if ((long long)n != sp.n) return fail(s, PIC_EINVAL, "n = %zu but the species holds %lld", n, sp.n);
    if (!x || !v) return fail(s, PIC_EINVAL, "null x or v");
    const bool bound = sp.d.kind == PIC_BOUND;
    if (bound && !xi) return fail(s, PIC_EINVAL, "bound species need xi");
    const bool dmpp = sp.d.kind == PIC_DIRAC && sp.d.mass_per_particle;
    if (dmpp && !xi) return fail(s, PIC_EINVAL, "per-carrier Dirac masses need xi[i][0]");
    const int dims = s->g.dims;
    std::vector<int> cell(n);
    std::vector<double> off[3], vv[3], xx[3];
    for (int a = 0; a < 3; ++a) { off[a].resize(n); vv[a].resize(n); xx[a].resize(bound || (dmpp && a == 0) ? n : 0); }
    for (size_t i = 0; i < n; ++i) {
        int c[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(x[3 * i + a]) || !std::isfinite(v[3 * i + a]) || (bound && !std::isfinite(xi[3 * i + a])))
                return fail(s, PIC_EINVAL, "non-finite input at particle %zu", i);
            vv[a][i] = v[3 * i + a];
            if (bound) xx[a][i] = xi[3 * i + a];
            if (a >= dims) continue;
            double X = x[3 * i + a] / s->g.dx[a];
            const double nn = (double)s->g.n[a];
            if (s->h.periodic[a]) {
                if (X >= nn) X -= nn;
                else if (X < 0.0) { X += nn; if (X >= nn) X = 0.0; }
            }
            double f = std::floor(X);
            double o = X - f;
            int ci = (int)f;
            if (o >= 1.0) { o = 0.0; ci += 1; }
            if (ci < 0 || ci >= s->g.n[a]) return fail(s, PIC_EINVAL, "particle %zu outside the grid", i);
            c[a] = ci;
            off[a][i] = o;
        }
        cell[i] = pack_cell(s->h, c[0], c[1], c[2]);
        if (dmpp) {
            const double m = xi[3 * i];
            if (!(m > 0.0) || !std::isfinite(m)) return fail(s, PIC_EINVAL, "Dirac mass of particle %zu must be positive", i);
            xx[0][i] = sp.d.q / m;  // stored as q / m_d
        }
    }
    const int p = sp.parity;
    HIPCHK(s, hipMemcpyAsync(sp.cell[p], cell.data(), n * sizeof(int), hipMemcpyHostToDevice, s->st));
    std::vector<char> buf;
    auto put = [&](void* dst, const std::vector<double>& src) -> hipError_t {
        if (s->es == 4) to_real<float>(src.data(), n, buf); else to_real<double>(src.data(), n, buf);
        hipError_t e = hipMemcpyAsync(dst, buf.data(), buf.size(), hipMemcpyHostToDevice, s->st);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s->st);
    };
    for (int a = 0; a < 3; ++a) {
        if (a < dims) HIPCHK(s, put(sp.off[p][a], off[a]));
        HIPCHK(s, put(sp.v[p][a], vv[a]));
        if (bound || (dmpp && a == 0)) HIPCHK(s, put(sp.xi[p][a], xx[a]));
    }
    HIPCHK(s, hipStreamSynchronize(s->st));
    s->need_sort = true;
    sp.sorted_once = false;
    return PIC_OK;
}

extern "C" int pic_load_fields(pic_sim* s, const double* e, const double* b)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind before loading fields");
    const size_t L = (size_t)s->h.Lvol;
    for (const double* src : {e, b})
        if (src)
            for (size_t q = 0; q < 3 * L; ++q)
                if (!std::isfinite(src[q])) return fail(s, PIC_EINVAL, "non-finite field value at entry %zu", q);
    std::vector<char> buf;
    for (int c = 0; c < 3; ++c) {
        for (int w = 0; w < 2; ++w) {
            const double* src = w == 0 ? e : b;
            if (!src) continue;
            if (s->es == 4) to_real<float>(src + c * L, L, buf); else to_real<double>(src + c * L, L, buf);
            const int par = (int)(s->step & 1);
            HIPCHK(s, hipMemcpyAsync(w == 0 ? s->h.E[par][c] : s->h.B[par][c], buf.data(), buf.size(), hipMemcpyHostToDevice, s->st));
            HIPCHK(s, hipStreamSynchronize(s->st));
        }
    }
    return PIC_OK;
}

extern "C" int pic_load_eps_inv(pic_sim* s, const double* einv)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind before loading the permittivity");
    if (s->batch_refs) return fail(s, PIC_ESTATE, "simulation is in a batch");
    if (!s->h.einv) return fail(s, PIC_EINVAL, "the grid was created with eps_cells = 0");
    if (!einv) return fail(s, PIC_EINVAL, "null einv");
    const size_t L = (size_t)s->h.Lvol;
    double mx = 0.0;
    for (size_t q = 0; q < 3 * L; ++q) {
        if (!(einv[q] > 0.0) || !std::isfinite(einv[q])) return fail(s, PIC_EINVAL, "einv entry %zu is not finite and positive", q);
        // the stored value must stay positive and finite in the working precision too
        if (s->es == 4 && !(einv[q] >= 1e-30 && einv[q] <= 1e30)) return fail(s, PIC_EINVAL, "einv entry %zu out of FP32 range", q);
        mx = std::max(mx, einv[q]);
    }
    if (int r = check_dt(s, nullptr, mx + s->eoff_max)) return r;
    std::vector<char> buf;
    if (s->es == 4) to_real<float>(einv, 3 * L, buf); else to_real<double>(einv, 3 * L, buf);
    HIPCHK(s, hipMemcpyAsync(s->h.einv, buf.data(), buf.size(), hipMemcpyHostToDevice, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    s->einv_max = mx;
    return PIC_OK;
}

extern "C" int pic_load_eps_offdiag(pic_sim* s, const double* e)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind before loading the permittivity");
    if (s->batch_refs) return fail(s, PIC_ESTATE, "simulation is in a batch");
    if (!s->h.eoff) return fail(s, PIC_EINVAL, "the grid was created without eps_cells = 2");
    if (!e) return fail(s, PIC_EINVAL, "null entries");
    const size_t L = (size_t)s->h.Lvol;
    const int L0 = s->h.L[0], L1 = s->h.L[1];
    double rowmax = 0.0;
    for (size_t q = 0; q < L; ++q) {
        const int g[3] = {(int)(q % L0), (int)((q / L0) % L1), (int)(q / ((size_t)L0 * L1))};
        // the averaged update terms must come from interior nodes: indices [2, n - 2] on open axes
        bool edge = false;
        for (int a = 0; a < s->g.dims; ++a)
            if (!s->h.periodic[a] && (g[a] < 2 || g[a] > s->h.n[a] - 2)) edge = true;
        for (int a = 0; a < 3; ++a) {
            double row = 0.0;
            for (int k = 0; k < 2; ++k) {
                const size_t i = (size_t)(2 * a + k) * L + q;
                const double v = e[i];
                if (!std::isfinite(v) || (s->es == 4 && !(std::fabs(v) < 1e30)))
                    return fail(s, PIC_EINVAL, "off-diagonal entry %zu is not finite", i);
                if (v != 0.0 && edge)
                    return fail(s, PIC_EINVAL, "off-diagonal entry %zu lies within two nodes of an open face", i);
                row += std::fabs(v);
            }
            rowmax = std::max(rowmax, row);
        }
    }
    if (int r = check_dt(s, nullptr, s->einv_max + rowmax)) return r;
    // the nodes with an off-diagonal row, and the nodes their averages read (+s e_a - t e_b)
    std::vector<char> need(L, 0);
    std::vector<int> lists(2 * L), counts(2, 0);
    for (size_t q = 0; q < L; ++q) {
        const int g[3] = {(int)(q % L0), (int)((q / L0) % L1), (int)(q / ((size_t)L0 * L1))};
        bool row = false;
        for (int m = 0; m < 6; ++m) {
            if (e[(size_t)m * L + q] == 0.0) continue;
            row = true;
            const int a = m / 2, b = (m % 2) < a ? (m % 2) : (m % 2) + 1;
            const int ns = a < s->g.dims ? 2 : 1, nt = b < s->g.dims ? 2 : 1;
            for (int sa = 0; sa < ns; ++sa)
                for (int tb = 0; tb < nt; ++tb) {
                    int h[3] = {g[0], g[1], g[2]};
                    h[a] += sa;
                    h[b] -= tb;
                    for (int x = 0; x < s->g.dims; ++x)
                        if (s->h.periodic[x]) h[x] = (h[x] % s->h.n[x] + s->h.n[x]) % s->h.n[x];
                    need[((size_t)h[2] * L1 + h[1]) * L0 + h[0]] = 1;
                }
        }
        if (row) lists[L + counts[1]++] = (int)q;
    }
    for (size_t q = 0; q < L; ++q)
        if (need[q]) lists[counts[0]++] = (int)q;
    std::vector<char> buf;
    if (s->es == 4) to_real<float>(e, 6 * L, buf); else to_real<double>(e, 6 * L, buf);
    HIPCHK(s, hipMemcpyAsync(s->h.eoff, buf.data(), buf.size(), hipMemcpyHostToDevice, s->st));
    HIPCHK(s, hipMemcpyAsync(s->h.tlist, lists.data(), lists.size() * sizeof(int), hipMemcpyHostToDevice, s->st));
    HIPCHK(s, hipMemcpyAsync(s->h.tcount, counts.data(), 2 * sizeof(int), hipMemcpyHostToDevice, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    s->eoff_max = rowmax;
    return PIC_OK;
}

extern "C" int pic_load_ext_field(pic_sim* s, const double* e)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind before loading the external field");
    if (s->batch_refs) return fail(s, PIC_ESTATE, "simulation is in a batch");
    if (!s->h.eext) return fail(s, PIC_EINVAL, "the grid was created with ext_field = 0");
    if (!e) return fail(s, PIC_EINVAL, "null field");
    const size_t L = (size_t)s->h.Lvol;
    for (size_t q = 0; q < 3 * L; ++q)
        if (!std::isfinite(e[q]) || (s->es == 4 && !(std::fabs(e[q]) < 3e38)))
            return fail(s, PIC_EINVAL, "external field entry %zu is not finite", q);
    std::vector<char> buf;
    if (s->es == 4) to_real<float>(e, 3 * L, buf); else to_real<double>(e, 3 * L, buf);
    HIPCHK(s, hipMemcpyAsync(s->h.eext, buf.data(), buf.size(), hipMemcpyHostToDevice, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return PIC_OK;
}

// charge density of the particles at the nodes, summed exactly (whole quanta and their fractions,
// as the current): the same for any order of the additions
static hipError_t launch_rho(pic_sim* s, double* rho)
{
    hipError_t e = enqueue_fill(rho, sizeof(double) * (size_t)s->h.Lvol, s->st);
    if (e == hipSuccess) e = enqueue_fill(s->h.rho_lo, sizeof(double) * (size_t)s->h.Lvol, s->st);
    if (e != hipSuccess) return e;
    if (s->g.precision == PIC_FP32) return Launchers<float>::rho(s->g.dims, dtab(s), rho, kDiagBlocks, s->st);
    return Launchers<double>::rho(s->g.dims, dtab(s), rho, kDiagBlocks, s->st);
}

extern "C" int pic_init_fields(pic_sim* s, int mode)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind first");
    if (s->batch_refs) return fail(s, PIC_ESTATE, "simulation is in a batch");
    if (mode < 0 || mode > 2) return fail(s, PIC_EINVAL, "mode");
    if (mode == 2 && !(s->g.dims == 1 && s->h.periodic[0])) return fail(s, PIC_EINVAL, "Gauss initialisation is 1D periodic only");
    HIPCHK(s, launch_rho(s, s->h.rho_a));
    if (mode == 0) {
        HIPCHK(s, enqueue_ion(s->d, s->h.rho_a, 0, nullptr, s->st));
    } else {
        HIPCHK(s, enqueue_sum(s->h.rho_a, s->h.Lvol, s->part, kDiagBlocks, s->st));
        HIPCHK(s, enqueue_final(s->part, kDiagBlocks, 1, 0, s->outv, s->st));
        HIPCHK(s, enqueue_ion(s->d, s->h.rho_a, 1, s->outv, s->st));
    }
    if (mode == 2) {
        const int par = (int)(s->step & 1);
        if (s->g.precision == PIC_FP32) HIPCHK(s, Launchers<float>::gauss_init_1d(s->d, par, s->h.rho_a, s->st));
        else HIPCHK(s, Launchers<double>::gauss_init_1d(s->d, par, s->h.rho_a, s->st));
    }
    HIPCHK(s, hipStreamSynchronize(s->st));
    return PIC_OK;
}

// ---------------------------------------------------------------------------------------------
// Step
// ---------------------------------------------------------------------------------------------
static int enqueue_sort_all(pic_sim* s, std::vector<int>* sorted)
{
    for (size_t i = 0; i < s->sp.size(); ++i) {
        SpeciesHost& x = s->sp[i];
        if (x.d.kind == PIC_BOUND && x.sorted_once) continue;  // anchors never move
        if (x.n > 0) {
            HIPCHK(s, enqueue_sort(s->d, (int)i, (int)x.n, s->passes, s->es, s->st));
            x.parity ^= 1;
        }
        HIPCHK(s, enqueue_ranges(s->d, (int)i, s->h.ntiles, s->passes, x.n > 0, s->st));
        x.sorted_once = true;
        if (sorted) sorted->push_back((int)i);
    }
    HIPCHK(s, enqueue_compact(s->d, s->h, s->st));
    s->need_sort = false;
    return PIC_OK;
}

// species options whose code lives only in the RARE particle kernels (the diffusive redraw)
static bool has_rare(const pic_sim* s)
{
    for (const auto& x : s->sp)
        if (x.d.reflect == 2) return true;
    return false;
}

// options whose extra loads live only in the EXT particle kernels: the static external field and
// the per-carrier Dirac mass
static bool has_extra(const pic_sim* s)
{
    if (s->h.eext) return true;
    for (const auto& x : s->sp)
        if (x.d.kind == PIC_DIRAC && x.d.mass_per_particle) return true;
    return false;
}

// the simulation's periodic active axes, a bit per axis (particle kernels are compiled for some masks)
static int sim_permask(const pic_sim* s)
{
    int m = 0;
    for (int a = 0; a < s->g.dims; ++a)
        if (s->h.periodic[a]) m |= 1 << a;
    return m;
}

static Launch make_launch(pic_sim* s)
{
    Launch L{};
    L.sims = s->d;
    L.nsims = 1;
    L.max_vf = s->h.Vf;
    L.max_vj = s->h.Vj;
    L.pgrid = s->pgrid;
    L.block = s->g.block;
    L.ftiles_total = s->h.nftiles;
    L.eps = s->h.einv != nullptr;
    L.rare = has_rare(s);
    L.ext = has_extra(s);
    L.tensor_lvol = s->h.eoff ? s->h.Lvol : 0;
    for (int a = 0; a < 3; ++a) L.tile[a] = s->h.T[a];
    L.permask = sim_permask(s);
    L.queue = s->pqueue;
    L.ncu = s->ncu;
    L.stream = s->st;
    return L;
}

static int enqueue_push_fields(pic_sim* s)
{
    const Launch L = make_launch(s);
    if (s->g.precision == PIC_FP32) {
        HIPCHK(s, Launchers<float>::particles(s->g.dims, L));
        HIPCHK(s, Launchers<float>::fields(s->g.dims, L, s->field_lds));
    } else {
        HIPCHK(s, Launchers<double>::particles(s->g.dims, L));
        HIPCHK(s, Launchers<double>::fields(s->g.dims, L, s->field_lds));
    }
    return PIC_OK;
}

static int enqueue_one_step(pic_sim* s)
{
    int r;
    if (s->need_sort || s->step % s->g.sort_every == 0)
        if ((r = enqueue_sort_all(s, nullptr))) return r;
    if (s->h.track) HIPCHK(s, launch_rho(s, s->h.rho_a));
    if ((r = enqueue_push_fields(s))) return r;
    if (s->h.track) {
        HIPCHK(s, launch_rho(s, s->h.rho_b));
        if (s->g.precision == PIC_FP32) HIPCHK(s, Launchers<float>::continuity(s->g.dims, s->d, s->part, kDiagBlocks, s->st));
        else HIPCHK(s, Launchers<double>::continuity(s->g.dims, s->d, s->part, kDiagBlocks, s->st));
        HIPCHK(s, enqueue_final(s->part, kDiagBlocks, 2, 1, s->cont, s->st));
    }
    s->step++;
    return PIC_OK;
}

static void drop_graph(pic_sim* s)
{
    if (s->gexec) {
        (void)hipGraphExecDestroy(s->gexec);
        s->gexec = nullptr;
    }
}

extern "C" int pic_use_graphs(pic_sim* s, int on)
{
    if (!s) return PIC_EINVAL;
    s->graphs = on != 0;
    if (!s->graphs) drop_graph(s);
    return PIC_OK;
}

// capture one sort period (sort + sort_every steps) starting at a multiple of sort_every
static int capture_period(pic_sim* s)
{
    drop_graph(s);
    const long long step0 = s->step;
    std::vector<int> par;
    for (auto& x : s->sp) par.push_back(x.parity);
    if (!s->st) return fail(s, PIC_EINVAL, "graphs need a non-default stream");
    HIPCHK(s, hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
    int r = PIC_OK;
    s->graph_species.clear();
    r = enqueue_sort_all(s, &s->graph_species);
    for (int k = 0; k < s->g.sort_every && !r; ++k) r = enqueue_push_fields(s);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s->st, &graph);
    // capture does not execute: restore the host view of the state
    s->step = step0;
    for (size_t i = 0; i < s->sp.size(); ++i) s->sp[i].parity = par[i];
    if (r) { if (graph) (void)hipGraphDestroy(graph); return r; }
    if (e != hipSuccess) return fail(s, PIC_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&s->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) { s->gexec = nullptr; return fail(s, PIC_EDEVICE, "graph instantiate: %s", hipGetErrorString(e)); }
    return PIC_OK;
}

extern "C" int pic_step(pic_sim* s, int nsteps)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind before stepping");
    if (s->batch_refs) return fail(s, PIC_ESTATE, "simulation is in a batch; use pic_batch_step");
    if (nsteps < 0) return fail(s, PIC_EINVAL, "nsteps");
    int r;
    while (nsteps > 0) {
        const int P = s->g.sort_every;
        const bool bound_sorted = [&] {
            for (auto& x : s->sp) if (x.d.kind == PIC_BOUND && !x.sorted_once) return false;
            return true;
        }();
        if (s->graphs && s->st && !s->h.track && !s->need_sort && bound_sorted && s->step % P == 0 && nsteps >= P) {
            if (!s->gexec && (r = capture_period(s))) return r;
            HIPCHK(s, hipGraphLaunch(s->gexec, s->st));
            for (int i : s->graph_species) s->sp[i].parity ^= 1;
            s->step += P;
            nsteps -= P;
            continue;
        }
        if ((r = enqueue_one_step(s))) return r;
        --nsteps;
    }
    return PIC_OK;
}

extern "C" int pic_time_kernels(pic_sim* s, int nsteps, double out[4])
{
    if (!s || !out) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind first");
    if (s->batch_refs) return fail(s, PIC_ESTATE, "simulation is in a batch");
    if (nsteps < 0) return PIC_EINVAL;
    // five events per step (sort start/end, particles start, fields start, fields end), all
    // recorded back to back on the simulation's stream and read after one synchronisation, so
    // that no host round trip falls between a kernel and its events
    std::vector<hipEvent_t> ev((size_t)5 * nsteps, nullptr);
    std::vector<char> sorted((size_t)nsteps, 0);
    int r = PIC_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) { r = fail(s, PIC_EDEVICE, "event create"); break; }
    for (int k = 0; k < nsteps && !r; ++k) {
        hipEvent_t* e = &ev[(size_t)5 * k];
        const bool sort = s->need_sort || s->step % s->g.sort_every == 0;
        hipError_t x = hipSuccess;
        if (sort) {
            sorted[k] = 1;
            x = hipEventRecord(e[0], s->st);
            if (x == hipSuccess && (r = enqueue_sort_all(s, nullptr))) break;
            if (x == hipSuccess) x = hipEventRecord(e[1], s->st);
        }
        const Launch L = make_launch(s);
        if (x == hipSuccess) x = hipEventRecord(e[2], s->st);
        if (x == hipSuccess) x = s->g.precision == PIC_FP32 ? Launchers<float>::particles(s->g.dims, L)
                                                            : Launchers<double>::particles(s->g.dims, L);
        if (x == hipSuccess) x = hipEventRecord(e[3], s->st);
        if (x == hipSuccess) x = s->g.precision == PIC_FP32 ? Launchers<float>::fields(s->g.dims, L, s->field_lds)
                                                            : Launchers<double>::fields(s->g.dims, L, s->field_lds);
        if (x == hipSuccess) x = hipEventRecord(e[4], s->st);
        if (x != hipSuccess) { r = fail(s, PIC_EDEVICE, "timing: %s", hipGetErrorString(x)); break; }
        s->step++;
    }
    double tp = 0.0, tf = 0.0, ts = 0.0;
    int nsort = 0;
    if (!r && hipStreamSynchronize(s->st) != hipSuccess) r = fail(s, PIC_EDEVICE, "timing sync");
    for (int k = 0; k < nsteps && !r; ++k) {
        hipEvent_t* e = &ev[(size_t)5 * k];
        float a = 0.f, b = 0.f, c = 0.f;
        (void)hipEventElapsedTime(&a, e[2], e[3]);
        (void)hipEventElapsedTime(&b, e[3], e[4]);
        tp += a;
        tf += b;
        if (sorted[k]) {
            (void)hipEventElapsedTime(&c, e[0], e[1]);
            ts += c;
            ++nsort;
        }
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (r) return r;
    out[0] = nsteps > 0 ? tp / nsteps : 0.0;
    out[1] = nsteps > 0 ? tf / nsteps : 0.0;
    out[2] = nsort > 0 ? ts / nsort : 0.0;
    out[3] = (double)nsort;
    return PIC_OK;
}

extern "C" int pic_sync(pic_sim* s)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return PIC_OK;
    HIPCHK(s, hipStreamSynchronize(s->st));
    return PIC_OK;
}

// ---------------------------------------------------------------------------------------------
// Diagnostics
// ---------------------------------------------------------------------------------------------
template <typename R>
static void from_real(const std::vector<char>& buf, size_t n, double* dst, size_t stride)
{
    const R* p = reinterpret_cast<const R*>(buf.data());
    for (size_t i = 0; i < n; ++i) dst[i * stride] = double(p[i]);
}

static int fetch_real(pic_sim* s, const void* src, size_t n, double* dst, size_t stride)
{
    std::vector<char> buf(n * s->es);
    if (n) {
        HIPCHK(s, hipMemcpyAsync(buf.data(), src, buf.size(), hipMemcpyDeviceToHost, s->st));
        HIPCHK(s, hipStreamSynchronize(s->st));
    }
    if (s->es == 4) from_real<float>(buf, n, dst, stride); else from_real<double>(buf, n, dst, stride);
    return PIC_OK;
}

static int fetch_doubles(pic_sim* s, const double* src, size_t n, double* dst)
{
    HIPCHK(s, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return PIC_OK;
}

extern "C" int pic_energy_histogram(pic_sim* s, int sid, double e_max, int nbins, uint64_t* counts)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind first");
    if (sid < 0 || sid >= (int)s->sp.size()) return fail(s, PIC_EINVAL, "species id");
    if (nbins < 1 || nbins > kMaxHistBins) return fail(s, PIC_EINVAL, "nbins must be 1 .. %d", kMaxHistBins);
    if (!(e_max > 0.0) || !std::isfinite(e_max)) return fail(s, PIC_EINVAL, "e_max must be positive");
    if (!counts) return fail(s, PIC_EINVAL, "null counts");
    HIPCHK(s, enqueue_fill(s->h.hist, sizeof(unsigned long long) * (size_t)(nbins + 1), s->st));
    if (s->sp[sid].n > 0) {
        if (s->es == 4) HIPCHK(s, Launchers<float>::energy_hist(dtab(s), sid, e_max, nbins, s->h.hist, s->st));
        else HIPCHK(s, Launchers<double>::energy_hist(dtab(s), sid, e_max, nbins, s->h.hist, s->st));
    }
    HIPCHK(s, hipMemcpyAsync(counts, s->h.hist, sizeof(unsigned long long) * (size_t)(nbins + 1),
                             hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return PIC_OK;
}

// ---------------------------------------------------------------------------------------------
// Histogram counts in a static device array, for callers that cannot allocate device memory.
// Each GPU the library runs on holds its own copy of `scratch` until the process ends; host code
// uses the device address hipGetSymbolAddress returns for the GPU (looked up once per device, at
// pic_bind, with that device current), never the array's name.  Every call on one GPU shares that
// GPU's copy: it is cleared at the start of each call, and calls that overlap on one GPU race.
// ---------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned long long scratch[kMaxHistBins + 1];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// The device address of the current GPU's copy of scratch (dev is that GPU).
static int scratch_address(pic_sim* s, int dev, unsigned long long** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(s, PIC_EDEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(s, PIC_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned long long*>(p);
    }
    *out = g_scratch_ptr[dev];
    return PIC_OK;
}

extern "C" int pic_energy_histogram_static(pic_sim* s, int sid, double e_max, int nbins, uint64_t* counts)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind first");
    if (sid < 0 || sid >= (int)s->sp.size()) return fail(s, PIC_EINVAL, "species id");
    if (nbins < 1 || nbins > kMaxHistBins)
        return fail(s, PIC_EINVAL, "nbins must be 1 .. %d (the static scratch holds %d counts)", kMaxHistBins,
                    kMaxHistBins + 1);
    if (!(e_max > 0.0) || !std::isfinite(e_max)) return fail(s, PIC_EINVAL, "e_max must be positive");
    if (!counts) return fail(s, PIC_EINVAL, "null counts");
    unsigned long long* scr = nullptr;
    if (int r = scratch_address(s, s->device, &scr)) return r;
    // zero fill by kernel (no memset node if the caller captures the stream)
    HIPCHK(s, enqueue_fill(scr, sizeof(unsigned long long) * (size_t)(nbins + 1), s->st));
    if (s->sp[sid].n > 0) {
        if (s->es == 4) HIPCHK(s, Launchers<float>::energy_hist(dtab(s), sid, e_max, nbins, scr, s->st));
        else HIPCHK(s, Launchers<double>::energy_hist(dtab(s), sid, e_max, nbins, scr, s->st));
    }
    HIPCHK(s, hipMemcpyAsync(counts, scr, sizeof(unsigned long long) * (size_t)(nbins + 1), hipMemcpyDeviceToHost,
                             s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return PIC_OK;
}

extern "C" int pic_diag(pic_sim* s, int kind, int arg, double* out, size_t cap, size_t* n_out)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "bind first");
    HIPCHK(s, hipStreamSynchronize(s->st));
    const bool f32 = s->g.precision == PIC_FP32;
    const size_t L = (size_t)s->h.Lvol;
    const int nsp = (int)s->sp.size();
    const int par = (int)(s->step & 1);  // field buffer holding the current E, B
    size_t need = 0;
    switch (kind) {
    case PIC_DIAG_FIELD_ENERGY: case PIC_DIAG_STEP: case PIC_DIAG_OVERFLOW: case PIC_DIAG_NONFINITE_FLAG:
        need = 1;
        break;
    case PIC_DIAG_KINETIC_ENERGY: need = arg < 0 ? nsp : 1; break;
    case PIC_DIAG_GAUSS_RESIDUAL: case PIC_DIAG_CONTINUITY: need = 2; break;
    case PIC_DIAG_CURRENT_SERIES: need = 3 * (size_t)std::min<long long>(s->step, s->h.series_cap); break;
    case PIC_DIAG_PARTICLE_COUNT: need = nsp; break;
    case PIC_DIAG_EXPORT_PARTICLES: case PIC_DIAG_KEYS:
        if (arg < 0 || arg >= nsp) return fail(s, PIC_EINVAL, "species id");
        need = (kind == PIC_DIAG_KEYS ? 1 : 9) * (size_t)s->sp[arg].n;
        break;
    case PIC_DIAG_EXPORT_FIELDS: need = 6 * L; break;
    case PIC_DIAG_EXPORT_CURRENT:
        if (!s->h.track) return fail(s, PIC_EINVAL, "current export needs track_continuity");
        need = 3 * L;
        break;
    default: return fail(s, PIC_EINVAL, "unknown diagnostic %d", kind);
    }
    if (n_out) *n_out = need;
    if (!out || cap < need) return fail(s, PIC_ETRUNC, "output needs %zu values", need);
    switch (kind) {
    case PIC_DIAG_FIELD_ENERGY: {
        if (f32) HIPCHK(s, Launchers<float>::field_energy(dtab(s), par, s->part, kDiagBlocks, s->st));
        else HIPCHK(s, Launchers<double>::field_energy(dtab(s), par, s->part, kDiagBlocks, s->st));
        HIPCHK(s, enqueue_final(s->part, kDiagBlocks, 1, 0, s->outv, s->st));
        int r = fetch_doubles(s, s->outv, 1, out);
        if (r) return r;
        if (!std::isfinite(out[0])) return fail(s, PIC_ENONFINITE, "non-finite field energy");
        return PIC_OK;
    }
    case PIC_DIAG_KINETIC_ENERGY: {
        for (int i = 0; i < nsp; ++i) {
            if (arg >= 0 && i != arg) continue;
            if (f32) HIPCHK(s, Launchers<float>::kinetic(dtab(s), i, s->part, kDiagBlocks, s->st));
            else HIPCHK(s, Launchers<double>::kinetic(dtab(s), i, s->part, kDiagBlocks, s->st));
            HIPCHK(s, enqueue_final(s->part, kDiagBlocks, 1, 0, s->outv, s->st));
            int r = fetch_doubles(s, s->outv, 1, out + (arg >= 0 ? 0 : i));
            if (r) return r;
            if (!std::isfinite(out[arg >= 0 ? 0 : i])) return fail(s, PIC_ENONFINITE, "non-finite kinetic energy");
        }
        return PIC_OK;
    }
    case PIC_DIAG_GAUSS_RESIDUAL: {
        HIPCHK(s, launch_rho(s, s->h.rho_b));
        if (f32) HIPCHK(s, Launchers<float>::gauss(s->g.dims, dtab(s), par, s->h.rho_b, s->part, kDiagBlocks, s->st));
        else HIPCHK(s, Launchers<double>::gauss(s->g.dims, dtab(s), par, s->h.rho_b, s->part, kDiagBlocks, s->st));
        HIPCHK(s, enqueue_final(s->part, kDiagBlocks, 2, 1, s->outv, s->st));
        return fetch_doubles(s, s->outv, 2, out);
    }
    case PIC_DIAG_CONTINUITY: return fetch_doubles(s, s->cont, 2, out);
    case PIC_DIAG_CURRENT_SERIES: return need ? fetch_doubles(s, s->h.series, need, out) : PIC_OK;
    case PIC_DIAG_PARTICLE_COUNT:
        for (int i = 0; i < nsp; ++i) out[i] = (double)s->sp[i].n;
        return PIC_OK;
    case PIC_DIAG_STEP: out[0] = (double)s->step; return PIC_OK;
    case PIC_DIAG_OVERFLOW: {
        unsigned long long c = 0;
        HIPCHK(s, hipMemcpyAsync(&c, s->h.over_count, sizeof(c), hipMemcpyDeviceToHost, s->st));
        HIPCHK(s, hipStreamSynchronize(s->st));
        out[0] = (double)c;
        return PIC_OK;
    }
    case PIC_DIAG_NONFINITE_FLAG: {
        int f = 0;
        HIPCHK(s, hipMemcpyAsync(&f, s->h.nonfinite, sizeof(f), hipMemcpyDeviceToHost, s->st));
        HIPCHK(s, hipStreamSynchronize(s->st));
        out[0] = (double)f;
        return PIC_OK;
    }
    case PIC_DIAG_EXPORT_PARTICLES: {
        SpeciesHost& x = s->sp[arg];
        const size_t n = (size_t)x.n;
        const int p = x.parity;
        std::vector<int> cell(n);
        if (n) {
            HIPCHK(s, hipMemcpyAsync(cell.data(), x.cell[p], n * sizeof(int), hipMemcpyDeviceToHost, s->st));
            HIPCHK(s, hipStreamSynchronize(s->st));
        }
        double* X = out;
        double* V = out + 3 * n;
        double* XI = out + 6 * n;
        std::fill(out, out + 9 * n, 0.0);
        int r;
        for (int a = 0; a < 3; ++a) {
            if (a < s->g.dims && (r = fetch_real(s, x.off[p][a], n, X + a, 3))) return r;
            if ((r = fetch_real(s, x.v[p][a], n, V + a, 3))) return r;
            if (x.d.kind == PIC_BOUND && (r = fetch_real(s, x.xi[p][a], n, XI + a, 3))) return r;
        }
        if (x.d.kind == PIC_DIRAC && x.d.mass_per_particle) {
            if ((r = fetch_real(s, x.xi[p][0], n, XI, 3))) return r;
            for (size_t i = 0; i < n; ++i) XI[3 * i] = x.d.q / XI[3 * i];  // stored q / m_d -> m_d
        }
        for (size_t i = 0; i < n; ++i) {
            int c[3];
            unpack_cell(s->h, cell[i], c);
            for (int a = 0; a < 3; ++a)
                X[3 * i + a] = a < s->g.dims ? ((double)c[a] + X[3 * i + a]) * s->g.dx[a] : 0.0;
        }
        return PIC_OK;
    }
    case PIC_DIAG_EXPORT_FIELDS: {
        int r;
        for (int c = 0; c < 3; ++c) {
            if ((r = fetch_real(s, s->h.E[par][c], L, out + c * L, 1))) return r;
            if ((r = fetch_real(s, s->h.B[par][c], L, out + (3 + c) * L, 1))) return r;
        }
        return PIC_OK;
    }
    case PIC_DIAG_EXPORT_CURRENT: {
        int r;
        for (int c = 0; c < 3; ++c)
            if ((r = fetch_real(s, static_cast<char*>(s->h.jtrack) + c * L * s->es, L, out + c * L, 1))) return r;
        return PIC_OK;
    }
    case PIC_DIAG_KEYS: {
        const size_t n = (size_t)s->sp[arg].n;
        std::vector<int> k(n);
        HIPCHK(s, enqueue_keys_only(dtab(s), arg, (int)n, s->st));
        if (n) {
            HIPCHK(s, hipMemcpyAsync(k.data(), s->h.sp[arg].keys, n * sizeof(int), hipMemcpyDeviceToHost, s->st));
            HIPCHK(s, hipStreamSynchronize(s->st));
        }
        for (size_t i = 0; i < n; ++i) out[i] = (double)k[i];
        return PIC_OK;
    }
    }
    return PIC_EINVAL;
}

extern "C" const char* pic_last_error(const pic_sim* s)
{
    return s ? s->err.c_str() : g_create_err.c_str();
}

extern "C" int pic_set_stream(pic_sim* s, void* hip_stream)
{
    if (!s) return PIC_EINVAL;
    if (!s->bound) return fail(s, PIC_ESTATE, "simulation is not bound");
    if (s->batch_refs) return fail(s, PIC_ESTATE, "simulation is in a batch");
    hipStream_t ns = reinterpret_cast<hipStream_t>(hip_stream);
    if (ns == s->st) return PIC_OK;
    // the new stream waits for everything enqueued on the old one so far
    hipEvent_t ev = nullptr;
    HIPCHK(s, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, s->st);
    if (e == hipSuccess) e = hipStreamWaitEvent(ns, ev, 0);
    (void)hipEventDestroy(ev);
    HIPCHK(s, e);
    s->st = ns;
    return PIC_OK;
}

extern "C" void pic_destroy(pic_sim* s)
{
    if (!s) return;
    if (s->batch_refs && s->owner) (void)pic_batch_remove(s->owner, s);
    drop_graph(s);
    delete s;
}

// ---------------------------------------------------------------------------------------------
// Batched form, over fixed slots.  The step graph (sort_every x (one particle launch + one field
// launch) over every slot of the table) is captured once; an empty slot holds an entry with no
// tiles and no units, which the kernels pass over.  A member's sorts are captured into a graph of
// its own when it joins.  Joining and leaving write one table entry on the batch stream, by a
// kernel (the host never waits for the device), and the step graph is captured again only when a
// joining member needs more than it was captured for: larger LDS windows or block, a kernel
// variant, or the full-tensor passes of a member (whose launches the graph holds per slot).
// ---------------------------------------------------------------------------------------------
static_assert(sizeof(SimDev) % 4 == 0, "table entries are copied as 32-bit words");
constexpr size_t kIdleBytes = 256;  // the counters an empty slot's entry points at

__global__ void k_put_entry(SimDev* dst, SimDev v)
{
    const unsigned* src = reinterpret_cast<const unsigned*>(&v);
    unsigned* d = reinterpret_cast<unsigned*>(dst);
    for (int i = threadIdx.x; i < (int)(sizeof(SimDev) / 4); i += blockDim.x) d[i] = src[i];
}

// write a table entry on a stream (the entry travels as a kernel argument)
static hipError_t put_entry(SimDev* dst, const SimDev& v, hipStream_t st)
{
    hipLaunchKernelGGL(k_put_entry, dim3(1), dim3(256), 0, st, dst, v);
    return hipGetLastError();
}

struct pic_batch {
    int max_sims = 0, dims = 0, precision = 0;
    SimDev* table = nullptr;          // device [max_sims]
    void* idle = nullptr;             // device: the counters of an empty slot's entry (zeroed)
    hipStream_t st = nullptr;
    std::vector<pic_sim*> slot;       // [max_sims]: the member in each slot, or null
    int size = 0;
    int period = 0;                   // the members' common sort period
    int ncu = 256;
    std::string err;
    hipGraphExec_t gexec = nullptr;   // the step graph
    int captures = 0;                 // how often the step graph was captured
    // what the step graph was captured for
    int g_vf = 0, g_vj = 0, g_block = 0, g_flds = 0;
    int g_tile[3] = {0, 0, 0};        // the members' common particle tile (0: they differ)
    int g_permask = -1;               // the members' common periodic active axes (-1: they differ)
    bool g_eps = false, g_rare = false, g_ext = false;
    std::vector<int> g_tensor;        // slots whose full-tensor passes it launches
    // sort graphs of members that left, released once the work enqueued before their leaving is done
    std::vector<std::pair<hipGraphExec_t, hipEvent_t>> retired;
};

static int bfail(pic_batch* b, int code, const char* msg)
{
    if (b) b->err = msg;
    return code;
}

// the batch's particle-kernel unit queue: in the zeroed counter block after the idle entry's words
static unsigned* batch_queue(const pic_batch* b)
{
    static_assert(64 + sizeof(unsigned) * kUnitQueueWords <= kIdleBytes, "queue in the counter block");
    return reinterpret_cast<unsigned*>(static_cast<char*>(b->idle) + 64);
}

static SimDev idle_entry(const pic_batch* b)
{
    SimDev e{};
    e.dims = b->dims;
    e.precision = b->precision;
    long long* w = reinterpret_cast<long long*>(b->idle);
    e.n_units = reinterpret_cast<int*>(w);  // no units
    e.step_p = w + 1;
    e.step_f = w + 2;
    return e;
}

static size_t batch_table_bytes(int max_sims)
{
    return (sizeof(SimDev) * (size_t)max_sims + kAlign - 1) / kAlign * kAlign;
}

extern "C" int pic_batch_footprint(int max_sims, int dims, size_t* bytes)
{
    if (!bytes || max_sims < 1 || max_sims > MAX_BATCH || dims < 1 || dims > 3) return PIC_EINVAL;
    *bytes = batch_table_bytes(max_sims) + kIdleBytes;
    return PIC_OK;
}

extern "C" int pic_batch_create(int max_sims, int dims, int precision, void* dev_arena, size_t bytes,
                                void* hip_stream, pic_batch** out)
{
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    size_t need = 0;
    if (pic_batch_footprint(max_sims, dims, &need)) return PIC_EINVAL;
    if (!dev_arena || bytes < need || reinterpret_cast<uintptr_t>(dev_arena) % kAlign) return PIC_ENOMEM;
    if (precision != PIC_FP32 && precision != PIC_FP64) return PIC_EINVAL;
    if (!hip_stream) return PIC_EINVAL;  // a batch is captured into graphs: not the legacy stream
    pic_batch* b = new (std::nothrow) pic_batch();
    if (!b) return PIC_ENOMEM;
    b->max_sims = max_sims;
    b->dims = dims;
    b->precision = precision;
    b->table = reinterpret_cast<SimDev*>(dev_arena);
    b->idle = reinterpret_cast<char*>(dev_arena) + batch_table_bytes(max_sims);
    b->st = reinterpret_cast<hipStream_t>(hip_stream);
    b->slot.assign(max_sims, nullptr);
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
        b->ncu = v;
    hipError_t e = enqueue_fill(b->idle, kIdleBytes, b->st);
    const SimDev idle = idle_entry(b);
    for (int i = 0; i < max_sims && e == hipSuccess; ++i) e = put_entry(b->table + i, idle, b->st);
    if (e != hipSuccess) {
        delete b;
        return PIC_EDEVICE;
    }
    *out = b;
    return PIC_OK;
}

static void batch_drop_graph(pic_batch* b)
{
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
}

// release the sort graphs of members that left once the device has passed their leaving
static void batch_reap(pic_batch* b, bool wait)
{
    size_t k = 0;
    for (auto& r : b->retired) {
        if (wait || hipEventQuery(r.second) == hipSuccess) {
            if (wait) (void)hipEventSynchronize(r.second);
            (void)hipGraphExecDestroy(r.first);
            (void)hipEventDestroy(r.second);
        } else {
            b->retired[k++] = r;
        }
    }
    b->retired.resize(k);
}

// does the step graph cover member s (its windows, block, kernel variants, no tensor passes)?
static bool graph_covers(const pic_batch* b, const pic_sim* s)
{
    // a graph captured with a fixed-shape kernel takes members of that shape and periodic axes
    const bool tile_ok = b->g_tile[0] == 0 ||
                         (b->g_tile[0] == s->h.T[0] && b->g_tile[1] == s->h.T[1] && b->g_tile[2] == s->h.T[2] &&
                          (b->g_permask < 0 || b->g_permask == sim_permask(s)));
    return b->gexec && tile_ok && s->h.Vf <= b->g_vf && s->h.Vj <= b->g_vj && s->g.block <= b->g_block &&
           s->field_lds <= b->g_flds && (!s->h.einv || b->g_eps) && (!has_rare(s) || b->g_rare) &&
           (!has_extra(s) || b->g_ext) && !s->h.eoff;
}

extern "C" int pic_batch_add(pic_batch* b, pic_sim* s)
{
    if (!b || !s) return PIC_EINVAL;
    if (!s->bound) return bfail(b, PIC_ESTATE, "simulation is not bound");
    if (s->batch_refs) return bfail(b, PIC_ESTATE, "simulation already in a batch");
    if (b->size >= b->max_sims) return bfail(b, PIC_ENOMEM, "batch is full");
    if (s->g.dims != b->dims || s->g.precision != b->precision) return bfail(b, PIC_EINVAL, "dims or precision differ");
    if (b->size > 0 && s->g.sort_every != b->period) return bfail(b, PIC_EINVAL, "members must share the sort period");
    if (s->h.track) return bfail(b, PIC_EINVAL, "continuity tracking is not batched");
    if (s->step % s->g.sort_every != 0) return bfail(b, PIC_ESTATE, "member must be at a multiple of its sort period");
    if (s->st != b->st) return bfail(b, PIC_EINVAL, "member must be bound to the batch stream");
    int i = 0;
    while (b->slot[i]) ++i;
    // first sort (bound species) outside the member's sort graph, on its own table
    if (s->need_sort || [&] { for (auto& x : s->sp) if (!x.sorted_once) return true; return false; }()) {
        if (enqueue_sort_all(s, nullptr)) return bfail(b, PIC_EDEVICE, s->err.c_str());
    }
    SimDev* entry = b->table + i;
    for (size_t j = 0; j < s->sp.size(); ++j) mirror_species(s, (int)j);
    if (put_entry(entry, s->h, b->st) != hipSuccess) return bfail(b, PIC_EDEVICE, "table entry write failed");
    // the member's periodic sorts, captured against its slot's entry (the host parities are put back:
    // each launch of the graph flips them)
    std::vector<int> par, sorted;
    for (auto& x : s->sp) par.push_back(x.parity);
    if (hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bfail(b, PIC_EDEVICE, "sort capture failed");
    SimDev* own = s->d;
    s->d = entry;
    const int r = enqueue_sort_all(s, &sorted);
    s->d = own;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->st, &graph);
    for (size_t j = 0; j < s->sp.size(); ++j) s->sp[j].parity = par[j];
    hipGraphExec_t gx = nullptr;
    if (!r && e == hipSuccess) e = hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (r || e != hipSuccess) {
        (void)put_entry(entry, idle_entry(b), b->st);
        return bfail(b, PIC_EDEVICE, r ? s->err.c_str() : hipGetErrorString(e));
    }
    s->bsort = gx;
    s->graph_species = sorted;
    s->batch_refs = 1;
    s->d_batch = entry;
    s->bslot = i;
    s->owner = b;
    b->slot[i] = s;
    if (b->size++ == 0) b->period = s->g.sort_every;
    if (!graph_covers(b, s)) batch_drop_graph(b);
    return PIC_OK;
}

extern "C" int pic_batch_remove(pic_batch* b, pic_sim* s)
{
    if (!b || !s) return PIC_EINVAL;
    if (!s->batch_refs || s->bslot < 0 || s->bslot >= b->max_sims || b->slot[s->bslot] != s)
        return bfail(b, PIC_EINVAL, "not a member");
    const int i = s->bslot;
    if (put_entry(b->table + i, idle_entry(b), b->st) != hipSuccess) return bfail(b, PIC_EDEVICE, "table entry write failed");
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, b->st) != hipSuccess)
        return bfail(b, PIC_EDEVICE, "event failed");
    b->retired.push_back({s->bsort, ev});
    s->bsort = nullptr;
    b->slot[i] = nullptr;
    --b->size;
    if (s->h.eoff) batch_drop_graph(b);  // the graph launches this slot's tensor passes
    s->batch_refs = 0;
    s->d_batch = nullptr;
    s->bslot = -1;
    s->owner = nullptr;
    // the member's own table from the host state (pointer parities), after its last batched step
    for (size_t j = 0; j < s->sp.size(); ++j) mirror_species(s, (int)j);
    if (put_entry(s->d, s->h, s->st) != hipSuccess) return bfail(b, PIC_EDEVICE, "table entry write failed");
    batch_reap(b, false);
    return PIC_OK;
}

extern "C" int pic_batch_size(const pic_batch* b) { return b ? b->size : 0; }

extern "C" int pic_batch_captures(const pic_batch* b) { return b ? b->captures : 0; }

extern "C" const char* pic_batch_last_error(const pic_batch* b) { return b ? b->err.c_str() : ""; }

extern "C" void pic_batch_destroy(pic_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->st);
    batch_drop_graph(b);
    batch_reap(b, true);
    for (auto* s : b->slot) {
        if (!s) continue;
        if (s->bsort) (void)hipGraphExecDestroy(s->bsort);
        s->bsort = nullptr;
        s->batch_refs = 0;
        s->d_batch = nullptr;
        s->bslot = -1;
        s->owner = nullptr;
        for (size_t j = 0; j < s->sp.size(); ++j) mirror_species(s, (int)j);
        (void)put_entry(s->d, s->h, s->st);
    }
    (void)hipStreamSynchronize(b->st);
    delete b;
}

// capture the step graph for the current members (with room for every slot)
static int batch_capture(pic_batch* b)
{
    batch_drop_graph(b);
    b->g_vf = b->g_vj = 1;
    b->g_block = 64;
    b->g_flds = 1;
    b->g_eps = b->g_rare = b->g_ext = false;
    b->g_tensor.clear();
    bool first = true;
    for (int i = 0; i < b->max_sims; ++i) {
        const pic_sim* s = b->slot[i];
        if (!s) continue;
        for (int a = 0; a < 3; ++a) {
            if (first) b->g_tile[a] = s->h.T[a];
            else if (b->g_tile[a] != s->h.T[a]) b->g_tile[0] = b->g_tile[1] = b->g_tile[2] = 0;
        }
        if (first) b->g_permask = sim_permask(s);
        else if (b->g_permask != sim_permask(s)) b->g_permask = -1;
        first = false;
        b->g_vf = std::max(b->g_vf, s->h.Vf);
        b->g_vj = std::max(b->g_vj, s->h.Vj);
        b->g_block = std::max(b->g_block, s->g.block);
        b->g_flds = std::max(b->g_flds, s->field_lds);
        b->g_eps = b->g_eps || s->h.einv != nullptr;
        b->g_rare = b->g_rare || has_rare(s);
        b->g_ext = b->g_ext || has_extra(s);
        if (s->h.eoff) b->g_tensor.push_back(i);
    }
    Launch L{};
    L.sims = b->table;
    L.nsims = b->max_sims;
    L.max_vf = b->g_vf;
    L.max_vj = b->g_vj;
    L.pgrid = b->ncu * 8;             // enough blocks for a full batch; blocks without units return
    L.block = b->g_block;
    L.ftiles_total = 1 << 30;         // the largest field grid; tasks are taken in a loop
    L.eps = b->g_eps;
    L.rare = b->g_rare;
    L.ext = b->g_ext;
    for (int a = 0; a < 3; ++a) L.tile[a] = b->g_tile[a];
    L.permask = b->g_permask;
    L.queue = batch_queue(b);
    L.ncu = b->ncu;
    L.stream = b->st;
    const bool f32 = b->precision == PIC_FP32;
    if (hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bfail(b, PIC_EDEVICE, "capture failed");
    hipError_t e = hipSuccess;
    for (int k = 0; k < b->period && e == hipSuccess; ++k) {
        e = f32 ? Launchers<float>::particles(b->dims, L) : Launchers<double>::particles(b->dims, L);
        // members with a full tensor fold its off-diagonal part into their current first
        for (int i : b->g_tensor) {
            if (e != hipSuccess) break;
            const pic_sim* s = b->slot[i];
            e = f32 ? Launchers<float>::tensor(b->dims, b->table + i, s->h.Lvol, b->st)
                    : Launchers<double>::tensor(b->dims, b->table + i, s->h.Lvol, b->st);
        }
        if (e == hipSuccess)
            e = f32 ? Launchers<float>::fields(b->dims, L, b->g_flds) : Launchers<double>::fields(b->dims, L, b->g_flds);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->st, &graph);
    if (e == hipSuccess) e = ec;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        b->gexec = nullptr;
        return bfail(b, PIC_EDEVICE, hipGetErrorString(e));
    }
    ++b->captures;
    return PIC_OK;
}

extern "C" int pic_batch_step(pic_batch* b, int k)
{
    if (!b) return PIC_EINVAL;
    if (b->size == 0) return PIC_OK;
    const int P = b->period;
    if (k % P) return bfail(b, PIC_EINVAL, "k must be a multiple of the sort period");
    if (!b->gexec) {
        const int r = batch_capture(b);
        if (r) return r;
    }
    for (int it = 0; it < k / P; ++it) {
        for (auto* s : b->slot) {
            if (!s) continue;
            if (hipGraphLaunch(s->bsort, b->st) != hipSuccess) return bfail(b, PIC_EDEVICE, "sort graph launch failed");
            for (int j : s->graph_species) s->sp[j].parity ^= 1;
        }
        if (hipGraphLaunch(b->gexec, b->st) != hipSuccess) return bfail(b, PIC_EDEVICE, "graph launch failed");
        for (auto* s : b->slot)
            if (s) s->step += P;
    }
    batch_reap(b, false);
    return PIC_OK;
}

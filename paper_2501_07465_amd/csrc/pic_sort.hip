// pic_sort.hip -- cell sort of libpic: stable LSD radix sort of the int32 tile-major cell keys,
// permutation of the particle arrays, per-tile particle ranges and the active-tile list.
//
// Keys and permutation are bit-exact with a stable sort: each pass ranks equal digits in
// input order (wavefront multisplit with ballots, then waves in order, then blocks in order).
// All kernels read their arrays through the device SimDev table, so a captured graph stays
// valid when the array pointers are swapped after each sort.
#include "pic_dpp.h"
#include "pic_internal.h"
#include "pic_sort.h"

namespace pic {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortBlock = 1024;

// keys[i] = tile-major key of particle i's cell (anchor cell for bound particles); vals[i] = i
__global__ void k_keys(SimDev* __restrict__ S, int s)
{
    const SpeciesDev& sp = S->sp[s];
    const int n = sp.n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int c[3];
        unpack_cell(*S, sp.cell[i], c);
        sp.keys[i] = cell_key(*S, c);
        sp.vals[i] = i;
    }
}

// digit histogram per block: hist[d * nb + b]
__global__ void __launch_bounds__(kSortBlock) k_radix_hist(SimDev* __restrict__ S, int s, int pass, int ipb)
{
    __shared__ int h[kRadix];
    const SpeciesDev& sp = S->sp[s];
    const int* keys = (pass & 1) ? sp.keys_alt : sp.keys;
    const int n = sp.n;
    const int nb = (n + ipb - 1) / ipb;
    for (int i = threadIdx.x; i < kRadix; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int b = blockIdx.x;
    if (b < nb) {
        const int lo = b * ipb, hi = min(n, lo + ipb);
        const int shift = pass * kRadixBits;
        for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1);
    }
    __syncthreads();
    if (b < nb)
        for (int d = threadIdx.x; d < kRadix; d += blockDim.x) S->sort_hist[d * nb + b] = h[d];
}

// exclusive scan of hist[0 .. kRadix * nb) by one block.  Wave w owns a contiguous segment; its
// lanes read it 64 consecutive entries at a time (coalesced), kScanGroup rows in flight.  Pass 1
// sums each segment, pass 2 scans it row by row (DPP wavefront scan) with the segment's offset
// carried in.
constexpr int kScanThreads = 1024;
constexpr int kScanGroup = 16;

__global__ void __launch_bounds__(kScanThreads) k_radix_scan(SimDev* __restrict__ S, int s, int ipb)
{
    constexpr int NW = kScanThreads / 64;
    __shared__ int wsum[NW];
    const int n = S->sp[s].n;
    const int nb = (n + ipb - 1) / ipb;
    const int total = kRadix * nb;
    int* H = S->sort_hist;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per_w = (total + NW * 64 - 1) / (NW * 64) * 64;
    const int w0 = min(total, wave * per_w), w1 = min(total, w0 + per_w);
    int acc = 0;
    for (int g = w0; g < w1; g += 64 * kScanGroup) {
        int v[kScanGroup];
#pragma unroll
        for (int k = 0; k < kScanGroup; ++k) {
            const int i = g + k * 64 + lane;
            v[k] = i < w1 ? H[i] : 0;
        }
#pragma unroll
        for (int k = 0; k < kScanGroup; ++k) acc += v[k];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) wsum[wave] = acc;
    __syncthreads();
    int carry = 0;
    for (int w = 0; w < wave; ++w) carry += wsum[w];
    const unsigned msk = scan_masks(lane);
    for (int g = w0; g < w1; g += 64 * kScanGroup) {
        int v[kScanGroup];
#pragma unroll
        for (int k = 0; k < kScanGroup; ++k) {
            const int i = g + k * 64 + lane;
            v[k] = i < w1 ? H[i] : 0;
        }
#pragma unroll
        for (int k = 0; k < kScanGroup; ++k) {
            const int inc = seg_scan<int>(v[k], msk);
            const int i = g + k * 64 + lane;
            if (i < w1) H[i] = carry + inc - v[k];
            carry += __builtin_amdgcn_readlane(inc, 63);
        }
    }
}

// stable scatter of one pass
__global__ void __launch_bounds__(kSortBlock) k_radix_scatter(SimDev* __restrict__ S, int s, int pass, int ipb)
{
    __shared__ int running[kRadix];
    __shared__ int wcnt[kSortBlock / 64][kRadix];
    const SpeciesDev& sp = S->sp[s];
    const int* kin = (pass & 1) ? sp.keys_alt : sp.keys;
    const int* vin = (pass & 1) ? sp.vals_alt : sp.vals;
    int* kout = (pass & 1) ? sp.keys : sp.keys_alt;
    int* vout = (pass & 1) ? sp.vals : sp.vals_alt;
    const int n = sp.n;
    const int nb = (n + ipb - 1) / ipb;
    const int b = blockIdx.x;
    if (b >= nb) return;
    const int shift = pass * kRadixBits;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x / 64;
    for (int d = threadIdx.x; d < kRadix; d += blockDim.x) running[d] = S->sort_hist[d * nb + b];
    for (int i = threadIdx.x; i < nw * kRadix; i += blockDim.x) wcnt[i / kRadix][i % kRadix] = 0;
    __syncthreads();
    const int lo = b * ipb, hi = min(n, lo + ipb);
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int base = lo; base < hi; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const bool act = i < hi;
        int key = 0, val = 0, d = 0;
        if (act) {
            key = kin[i];
            val = vin[i];
            d = (key >> shift) & (kRadix - 1);
        }
        // lanes of this wave holding the same digit
        unsigned long long peers = __ballot(act);
#pragma unroll
        for (int bit = 0; bit < kRadixBits; ++bit) {
            const unsigned long long m = __ballot(act && ((d >> bit) & 1));
            peers &= ((d >> bit) & 1) ? m : ~m;
        }
        const int rank = __popcll(peers & lt);
        const int cnt = __popcll(peers);
        if (act && rank == 0) wcnt[wave][d] = cnt;
        __syncthreads();
        if (act) {
            int off = running[d] + rank;
            for (int w = 0; w < wave; ++w) off += wcnt[w][d];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        for (int dd = threadIdx.x; dd < kRadix; dd += blockDim.x) {
            int t = 0;
            for (int w = 0; w < nw; ++w) {
                t += wcnt[w][dd];
                wcnt[w][dd] = 0;
            }
            running[dd] += t;
        }
        __syncthreads();
    }
}

// After the last pass the sorted keys and the source index of each slot sit in keys/vals
// (even number of passes) or keys_alt/vals_alt (odd).  Gather every particle array into its
// alternate buffer.
__global__ void k_permute(SimDev* __restrict__ S, int s, int passes, int elem)
{
    const SpeciesDev& sp = S->sp[s];
    const int* perm = (passes & 1) ? sp.vals_alt : sp.vals;
    const int n = sp.n;
    const int dims = S->dims;
    const bool bound = sp.kind == BOUND;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int j = perm[i];
        sp.cell_alt[i] = sp.cell[j];
        if (elem == 4) {
            for (int a = 0; a < dims; ++a)
                reinterpret_cast<float*>(sp.off_alt[a])[i] = reinterpret_cast<const float*>(sp.off[a])[j];
            for (int a = 0; a < 3; ++a)
                reinterpret_cast<float*>(sp.v_alt[a])[i] = reinterpret_cast<const float*>(sp.v[a])[j];
            if (bound)
                for (int a = 0; a < 3; ++a)
                    reinterpret_cast<float*>(sp.xi_alt[a])[i] = reinterpret_cast<const float*>(sp.xi[a])[j];
        } else {
            for (int a = 0; a < dims; ++a)
                reinterpret_cast<double*>(sp.off_alt[a])[i] = reinterpret_cast<const double*>(sp.off[a])[j];
            for (int a = 0; a < 3; ++a)
                reinterpret_cast<double*>(sp.v_alt[a])[i] = reinterpret_cast<const double*>(sp.v[a])[j];
            if (bound)
                for (int a = 0; a < 3; ++a)
                    reinterpret_cast<double*>(sp.xi_alt[a])[i] = reinterpret_cast<const double*>(sp.xi[a])[j];
        }
    }
}

// Swap the particle arrays with their alternates (one thread).
__global__ void k_swap(SimDev* __restrict__ S, int s)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    SpeciesDev& sp = S->sp[s];
    int* c = sp.cell; sp.cell = sp.cell_alt; sp.cell_alt = c;
    for (int a = 0; a < 3; ++a) {
        void* t = sp.off[a]; sp.off[a] = sp.off_alt[a]; sp.off_alt[a] = t;
        t = sp.v[a]; sp.v[a] = sp.v_alt[a]; sp.v_alt[a] = t;
        t = sp.xi[a]; sp.xi[a] = sp.xi_alt[a]; sp.xi_alt[a] = t;
    }
}

// tile_start[t] = first sorted index whose key >= t * tile volume (lower bound), t = 0..ntiles
__global__ void k_tile_ranges(SimDev* __restrict__ S, int s, int passes)
{
    const SpeciesDev& sp = S->sp[s];
    const int* keys = (passes & 1) ? sp.keys_alt : sp.keys;
    const int n = sp.n;
    const int tvol = S->T[0] * S->T[1] * S->T[2];
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t <= S->ntiles; t += gridDim.x * blockDim.x) {
        const long long target = (long long)t * tvol;
        int lo = 0, hi = n;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((long long)keys[mid] < target) lo = mid + 1; else hi = mid;
        }
        sp.tile_start[t] = lo;
    }
}

// Active tiles (any species has particles) in tile order, and their work units: a tile holding
// c particles (all species) gets ceil(c / U) units of at most U particles, in its species-
// concatenated order (one unit when U is 0); the units of a tile take consecutive slots.
__global__ void __launch_bounds__(1024) k_compact(SimDev* __restrict__ S)
{
    __shared__ int wa[16], wu[16];
    const int nt = S->ntiles;
    const int U = S->unit_cap;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int per = (nt + blockDim.x - 1) / blockDim.x;
    const int lo = min(nt, tid * per), hi = min(nt, lo + per);
    auto count = [&](int t) {
        int c = 0;
        for (int s = 0; s < S->nspecies; ++s) c += S->sp[s].tile_start[t + 1] - S->sp[s].tile_start[t];
        return c;
    };
    auto nunits = [&](int c) { return c == 0 ? 0 : (U > 0 ? (c + U - 1) / U : 1); };
    int ca = 0, cu = 0;
    for (int t = lo; t < hi; ++t) {
        const int c = count(t);
        ca += c > 0 ? 1 : 0;
        cu += nunits(c);
    }
    // exclusive prefixes of the active-tile and unit counts over threads
    int ia = ca, iu = cu;
    for (int off = 1; off < 64; off <<= 1) {
        const int ta = __shfl_up(ia, off, 64), tu = __shfl_up(iu, off, 64);
        if (lane >= off) { ia += ta; iu += tu; }
    }
    if (lane == 63) { wa[wave] = ia; wu[wave] = iu; }
    __syncthreads();
    int ba = 0, bu = 0, ta = 0, tu = 0;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) { ba += wa[w]; bu += wu[w]; }
        ta += wa[w];
        tu += wu[w];
    }
    // a list that does not fit (particles in tiles the capacity did not count) is dropped whole
    // and flagged: no particle moves this period
    const bool fits = ta <= S->max_slots && tu <= S->max_units;
    int ra = ba + ia - ca, ru = bu + iu - cu;
    for (int t = lo; t < hi; ++t) {
        const int c = count(t);
        if (c > 0 && fits) {
            const int k = nunits(c);
            S->active[ra] = t;
            S->tile_slot[t] = ru;
            S->tile_nslot[t] = k;
            for (int j = 0; j < k; ++j) {
                int* u = S->units + 3 * (ru + j);
                u[0] = t;
                u[1] = U > 0 ? j * U : 0;
                u[2] = U > 0 ? min(c, (j + 1) * U) : c;
            }
            ++ra;
            ru += k;
        } else {
            S->tile_slot[t] = -1;
            S->tile_nslot[t] = 0;
        }
    }
    if (tid == 0) {
        *S->n_active = fits ? ta : 0;
        *S->n_units = fits ? tu : 0;
        if (!fits) atomicAdd(S->over_count, 1ull << 40);
    }
}

// --------------------------------------------------------------------------------------------
hipError_t enqueue_sort(SimDev* dS, int s, int n, int passes, int elem, hipStream_t st)
{
    const int ipb = sort_ipb(n);
    const int nb = (n + ipb - 1) / ipb;
    const int g = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    if (n > 0) {
        hipLaunchKernelGGL(k_keys, dim3(g > 0 ? g : 1), dim3(256), 0, st, dS, s);
        for (int p = 0; p < passes; ++p) {
            hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortBlock), 0, st, dS, s, p, ipb);
            hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(kScanThreads), 0, st, dS, s, ipb);
            hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kSortBlock), 0, st, dS, s, p, ipb);
        }
        hipLaunchKernelGGL(k_permute, dim3(g > 0 ? g : 1), dim3(256), 0, st, dS, s, passes, elem);
        hipLaunchKernelGGL(k_swap, dim3(1), dim3(64), 0, st, dS, s);
    }
    return hipGetLastError();
}

hipError_t enqueue_keys_only(SimDev* dS, int s, int n, hipStream_t st)
{
    const int g = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_keys, dim3(g > 0 ? g : 1), dim3(256), 0, st, dS, s);
    return hipGetLastError();
}

hipError_t enqueue_ranges(SimDev* dS, int s, int ntiles, int passes, hipStream_t st)
{
    const int g = (ntiles + 1 + 255) / 256;
    hipLaunchKernelGGL(k_tile_ranges, dim3(g), dim3(256), 0, st, dS, s, passes);
    return hipGetLastError();
}

hipError_t enqueue_compact(SimDev* dS, hipStream_t st)
{
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, dS);
    return hipGetLastError();
}

}  // namespace pic

namespace pic {

// ---- untyped helpers ---------------------------------------------------------------------------
__global__ void k_fill(unsigned* __restrict__ p, long long nwords)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nwords; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t enqueue_fill(void* p, size_t bytes, hipStream_t st)
{
    const long long nw = (long long)(bytes / 4);
    if (nw <= 0) return hipSuccess;
    long long g = (nw + 255) / 256;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(256), 0, st, reinterpret_cast<unsigned*>(p), nw);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_sum(const double* __restrict__ x, long long n, double* part)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) acc += x[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

hipError_t enqueue_sum(const double* x, long long n, double* part, int nb, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum, dim3(nb), dim3(256), 0, st, x, n, part);
    return hipGetLastError();
}

// out[v] = reduction over b of part[b * nv + v] in block order (op 0 sum, 1 max); one thread per v
__global__ void k_final(const double* __restrict__ part, int nb, int nv, int op, double* out)
{
    const int v = threadIdx.x;
    if (v >= nv) return;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double x = part[b * nv + v];
        acc = op ? fmax(acc, x) : acc + x;
    }
    out[v] = acc;
}

hipError_t enqueue_final(const double* part, int nb, int nv, int op, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_final, dim3(1), dim3(64), 0, st, part, nb, nv, op, out);
    return hipGetLastError();
}

// fixed ion background: -rho node by node, or minus the mean of rho (total / number of nodes)
__global__ void k_ion(SimDev* __restrict__ S, const double* __restrict__ rho, int uniform, const double* total)
{
    const double mean = uniform ? *total / (double)S->Lvol : 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < S->Lvol; q += (long long)gridDim.x * blockDim.x)
        S->rho_ion[q] = uniform ? -mean : -rho[q];
}

hipError_t enqueue_ion(SimDev* dS, const double* rho, int uniform, const double* total, hipStream_t st)
{
    hipLaunchKernelGGL(k_ion, dim3(1024), dim3(256), 0, st, dS, rho, uniform, total);
    return hipGetLastError();
}

}  // namespace pic

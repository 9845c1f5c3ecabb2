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
#include "pic.h"
#include "pic_measure.h"

namespace pic {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortBlock = 1024;
// the fused digit totals are spread over kPartCopies copies (block b adds into copy b % copies) so
// that fewer blocks queue on each address; the row scan sums the copies
constexpr int kPartCopies = 8;

// keys[i] = tile-major key of particle i's cell (anchor cell for bound particles).  The values the
// passes carry start as the identity, which the first scatter pass forms from the index (not stored).
// Block 0 also clears the digit totals the first histogram pass adds into.
__global__ void k_keys(SimDev* __restrict__ S, int s)
{
    const SpeciesDev& sp = S->sp[s];
    const int n = sp.n;
    if (blockIdx.x == 0)
        for (int d = threadIdx.x; d < kPartCopies * kRadix; d += blockDim.x) S->sort_part[d] = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int c[3];
        unpack_cell(*S, sp.cell[i], c);
        sp.keys[i] = cell_key(*S, c);
    }
}

// digit histogram per block: hist[d * nb + b].  For sorts of at most kFuseBlocks blocks the digit
// totals part[d] are summed here with one atomic per block and digit (part is zero on entry: cleared
// by k_keys, then by each scatter pass); larger sorts form them in k_radix_rowsum.
constexpr int kFuseBlocks = 1024;

__global__ void __launch_bounds__(kSortBlock) k_radix_hist(SimDev* __restrict__ S, int s, int pass, int ipb, int fuse)
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
        for (int d = threadIdx.x; d < kRadix; d += blockDim.x) {
            S->sort_hist[d * nb + b] = h[d];
            if (fuse && h[d]) atomicAdd(&S->sort_part[(b % kPartCopies) * kRadix + d], h[d]);
        }
}

// Exclusive scan of hist[0 .. kRadix * nb) (digit-major), one block per digit: each row scanned with
// its offset, the sum of the totals of the lower digits (the totals come from the histogram pass).
constexpr int kScanThreads = 1024;
constexpr int kUnitBlock = 4;  // tiles per active axis of a block of the unit list

// inclusive scan of v over the block (kScanThreads threads): DPP wavefront scans, then the wave
// totals in order; *total receives the block total
__device__ __forceinline__ int block_scan(int v, int* wsum, int* total)
{
    constexpr int NW = kScanThreads / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int inc = seg_scan<int>(v, scan_masks(lane));
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int carry = 0, all = 0;
    for (int w = 0; w < NW; ++w) {
        const int x = wsum[w];
        if (w < wave) carry += x;
        all += x;
    }
    __syncthreads();
    *total = all;
    return carry + inc;
}

// part[d] = sum over blocks b of hist[d * nb + b] (sorts of many blocks: the histogram pass's
// per-digit atomics would queue on 256 addresses)
__global__ void __launch_bounds__(kScanThreads) k_radix_rowsum(SimDev* __restrict__ S, int s, int ipb)
{
    __shared__ int wsum[kScanThreads / 64];
    const int n = S->sp[s].n;
    const int nb = (n + ipb - 1) / ipb;
    const int* row = S->sort_hist + (long long)blockIdx.x * nb;
    int acc = 0;
    for (int b = threadIdx.x; b < nb; b += kScanThreads) acc += row[b];
    int total;
    block_scan(acc, wsum, &total);
    if (threadIdx.x == 0) S->sort_part[blockIdx.x] = total;  // copy 0; the other copies stay zero
}

// row d of hist replaced by its exclusive prefix in the digit-major order: thread t scans its
// run of k consecutive entries serially, the runs are combined by one block scan
__global__ void __launch_bounds__(kScanThreads) k_radix_rowscan(SimDev* __restrict__ S, int s, int ipb)
{
    __shared__ int wsum[kScanThreads / 64];
    const int n = S->sp[s].n;
    const int nb = (n + ipb - 1) / ipb;
    const int d = blockIdx.x, tid = threadIdx.x;
    int total;
    int mine = 0;
    if (tid < d)
        for (int k = 0; k < kPartCopies; ++k) mine += S->sort_part[k * kRadix + tid];
    const int below = block_scan(mine, wsum, &total);
    (void)below;
    const int offset = total;  // sum of the totals of digits 0 .. d-1
    int* row = S->sort_hist + (long long)d * nb;
    const int k = (nb + kScanThreads - 1) / kScanThreads;
    const int b0 = min(nb, tid * k), b1 = min(nb, b0 + k);
    int run = 0;
    for (int b = b0; b < b1; ++b) run += row[b];
    const int inc = block_scan(run, wsum, &total);
    int acc = offset + inc - run;
    for (int b = b0; b < b1; ++b) {
        const int x = row[b];
        row[b] = acc;
        acc += x;
    }
}

// Stable scatter of one pass, in rounds of K keys per thread (key j of thread t in a round is the
// round's key j * kSortBlock + t, so the keys of a round are taken in input order item by item).
// Each wavefront ranks its lanes' equal digits with ballots and its first lane of each digit
// stores the count; one thread per digit then turns the (item, wave) counts of its digit, in
// input order, into the slot of each group's first key, and every key goes to that slot plus its
// rank.  Four barriers per round: K = 4 for blocks of at least 4096 keys, 1 for smaller ones.
template <int K>
__global__ void __launch_bounds__(kSortBlock) k_radix_scatter(SimDev* __restrict__ S, int s, int pass, int ipb)
{
    constexpr int NW = kSortBlock / 64;
    __shared__ int running[kRadix];
    __shared__ int wcnt[K][NW][kRadix];
    const SpeciesDev& sp = S->sp[s];
    const int* kin = (pass & 1) ? sp.keys_alt : sp.keys;
    const int* vin = (pass & 1) ? sp.vals_alt : sp.vals;
    int* kout = (pass & 1) ? sp.keys : sp.keys_alt;
    int* vout = (pass & 1) ? sp.vals : sp.vals_alt;
    const int n = sp.n;
    const int nb = (n + ipb - 1) / ipb;
    const int b = blockIdx.x;
    if (b >= nb) return;
    // the digit totals of this pass were consumed by the row scan: clear them for the next pass
    if (b == 0)
        for (int d = threadIdx.x; d < kPartCopies * kRadix; d += blockDim.x) S->sort_part[d] = 0;
    const int shift = pass * kRadixBits;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < kRadix; d += blockDim.x) running[d] = S->sort_hist[d * nb + b];
    const int lo = b * ipb, hi = min(n, lo + ipb);
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int base = lo; base < hi; base += K * kSortBlock) {
        for (int i = threadIdx.x; i < K * NW * kRadix; i += blockDim.x) (&wcnt[0][0][0])[i] = 0;
        int key[K], val[K], d[K], rank[K];
        bool act[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int i = base + j * kSortBlock + (int)threadIdx.x;
            act[j] = i < hi;
            key[j] = act[j] ? kin[i] : 0;
            val[j] = act[j] ? (pass == 0 ? i : vin[i]) : 0;  // the first pass carries each key's own index
            d[j] = (key[j] >> shift) & (kRadix - 1);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < K; ++j) {
            // lanes of this wave holding the same digit
            unsigned long long peers = __ballot(act[j]);
#pragma unroll
            for (int bit = 0; bit < kRadixBits; ++bit) {
                const unsigned long long m = __ballot(act[j] && ((d[j] >> bit) & 1));
                peers &= ((d[j] >> bit) & 1) ? m : ~m;
            }
            rank[j] = __popcll(peers & lt);
            if (act[j] && rank[j] == 0) wcnt[j][wave][d[j]] = __popcll(peers);
        }
        __syncthreads();
        for (int dd = threadIdx.x; dd < kRadix; dd += blockDim.x) {
            int acc = running[dd];
            for (int j = 0; j < K; ++j)
                for (int w = 0; w < NW; ++w) {
                    const int c = wcnt[j][w][dd];
                    wcnt[j][w][dd] = acc;
                    acc += c;
                }
            running[dd] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (act[j]) {
                const int off = wcnt[j][wave][d[j]] + rank[j];
                kout[off] = key[j];
                vout[off] = val[j];
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
            else if (sp.mpp)
                reinterpret_cast<float*>(sp.xi_alt[0])[i] = reinterpret_cast<const float*>(sp.xi[0])[j];
        } else {
            for (int a = 0; a < dims; ++a)
                reinterpret_cast<double*>(sp.off_alt[a])[i] = reinterpret_cast<const double*>(sp.off[a])[j];
            for (int a = 0; a < 3; ++a)
                reinterpret_cast<double*>(sp.v_alt[a])[i] = reinterpret_cast<const double*>(sp.v[a])[j];
            if (bound)
                for (int a = 0; a < 3; ++a)
                    reinterpret_cast<double*>(sp.xi_alt[a])[i] = reinterpret_cast<const double*>(sp.xi[a])[j];
            else if (sp.mpp)
                reinterpret_cast<double*>(sp.xi_alt[0])[i] = reinterpret_cast<const double*>(sp.xi[0])[j];
        }
    }
}

// tile_start[t] = first sorted index whose key >= t * tile volume (lower bound), t = 0..ntiles.
// After a sort (swap != 0) the first thread also swaps the particle arrays with their alternates,
// into which the permutation was gathered; nothing here reads them.
__global__ void k_tile_ranges(SimDev* __restrict__ S, int s, int passes, int swap)
{
    if (swap && blockIdx.x == 0 && threadIdx.x == 0) {
        SpeciesDev& w = S->sp[s];
        int* c = w.cell; w.cell = w.cell_alt; w.cell_alt = c;
        for (int a = 0; a < 3; ++a) {
            void* t = w.off[a]; w.off[a] = w.off_alt[a]; w.off_alt[a] = t;
            t = w.v[a]; w.v[a] = w.v_alt[a]; w.v_alt[a] = t;
            t = w.xi[a]; w.xi[a] = w.xi_alt[a]; w.xi_alt[a] = t;
        }
    }
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

// Active tiles (any species has particles) and their work units: a tile holding c particles (all
// species) gets ceil(c / U) units of at most U particles, in its species-concatenated order (one
// unit when U is 0); the units of a tile take consecutive slots.
//
// Tiles are listed in blocks of kUnitBlock tiles along each active axis (x fastest inside a block,
// blocks in x-fastest order), so that tiles near each other along every axis are near each other
// in the list, and the particle kernel, which takes units in list order on each XCD, processes them
// close together in time (their shared window halos meet in L2).  Ranks run over the grid of tiles
// padded to whole blocks; a rank whose tile lies beyond the grid is skipped.
//
// A list of one round is built by one block in one launch (k_compact_one).  Longer lists take
// three launches over rounds of kCompactK * 1024 ranks (each thread kCompactK consecutive ranks),
// each block of the first and last taking a contiguous run of rounds: k_compact_count forms each
// block's totals of active tiles and units, k_compact_scan their exclusive prefix in block order
// (and whether the lists fit), k_compact_place places the tiles and units of each round with a
// block scan from its block's prefix.  The block totals and prefixes live in sort_part, which every
// sort clears at its start.
constexpr int kCompactK = 4;
constexpr int kCompactBlocks = kPartCopies * kRadix / 2 - 1;  // block totals in sort_part (its last word: the fit flag)

struct CompactGeom {
    int sh[3], nb[3], vsh, nt, rounds, rpb;
    __device__ __forceinline__ explicit CompactGeom(const SimDev* S)
    {
        static_assert((kUnitBlock & (kUnitBlock - 1)) == 0 && kUnitBlock % kCompactK == 0, "blocks of whole thread runs");
        constexpr int kBS = kUnitBlock == 4 ? 2 : (kUnitBlock == 8 ? 3 : 1);  // log2 of kUnitBlock
        for (int a = 0; a < 3; ++a) {
            sh[a] = a < S->dims ? kBS : 0;
            nb[a] = (S->ntile[a] + (1 << sh[a]) - 1) >> sh[a];
        }
        vsh = sh[0] + sh[1] + sh[2];                 // log2 of the ranks per block
        nt = (nb[0] * nb[1] * nb[2]) << vsh;         // padded ranks
        rounds = (nt + kCompactK * kScanThreads - 1) / (kCompactK * kScanThreads);
        rpb = (rounds + gridDim.x - 1) / gridDim.x;  // rounds per block
    }
    // the tiles of ranks r .. r + kCompactK - 1 (-1 beyond the grid); they lie in one block of the
    // list (a block holds a multiple of kCompactK ranks), so its position is divided out once
    __device__ __forceinline__ void tiles_of(const SimDev* S, int r, int (&t)[kCompactK]) const
    {
        const int blk = r >> vsh;
        const int b1 = blk / nb[0];
        const int o0 = (blk - b1 * nb[0]) << sh[0];
        const int b2 = b1 / nb[1];
        const int o1 = (b1 - b2 * nb[1]) << sh[1], o2 = b2 << sh[2];
#pragma unroll
        for (int j = 0; j < kCompactK; ++j) {
            const int w = (r + j) & ((1 << vsh) - 1);
            const int c0 = o0 + (w & ((1 << sh[0]) - 1));
            const int c1 = o1 + ((w >> sh[0]) & ((1 << sh[1]) - 1));
            const int c2 = o2 + (w >> (sh[0] + sh[1]));
            t[j] = r + j < nt && c0 < S->ntile[0] && c1 < S->ntile[1] && c2 < S->ntile[2]
                       ? (c2 * S->ntile[1] + c1) * S->ntile[0] + c0
                       : -1;
        }
    }
};

__device__ __forceinline__ int compact_count(const SimDev* S, int t)
{
    int c = 0;
    for (int s = 0; s < S->nspecies; ++s) c += S->sp[s].tile_start[t + 1] - S->sp[s].tile_start[t];
    return c;
}
__device__ __forceinline__ int compact_units(const SimDev* S, int c)
{
    return c == 0 ? 0 : (S->unit_cap > 0 ? (c + S->unit_cap - 1) / S->unit_cap : 1);
}

__global__ void __launch_bounds__(kScanThreads) k_compact_count(SimDev* __restrict__ S)
{
    __shared__ int wsum[kScanThreads / 64];
    const CompactGeom G(S);
    int ca = 0, cu = 0;
    const int r0 = blockIdx.x * G.rpb, r1 = min(G.rounds, r0 + G.rpb);
    for (int round = r0; round < r1; ++round) {
        int t[kCompactK];
        G.tiles_of(S, round * kCompactK * kScanThreads + threadIdx.x * kCompactK, t);
#pragma unroll
        for (int j = 0; j < kCompactK; ++j) {
            const int c = t[j] >= 0 ? compact_count(S, t[j]) : 0;
            ca += c > 0 ? 1 : 0;
            cu += compact_units(S, c);
        }
    }
    int ta, tu;
    block_scan(ca, wsum, &ta);
    block_scan(cu, wsum, &tu);
    if (threadIdx.x == 0) {
        S->sort_part[2 * blockIdx.x] = ta;
        S->sort_part[2 * blockIdx.x + 1] = tu;
    }
}

// one block: the blocks' exclusive prefixes in place of their totals, the list lengths, and whether
// the lists fit (a list that does not fit, with particles in tiles the capacity did not count, is
// dropped whole and flagged: no particle moves this period)
__global__ void __launch_bounds__(kScanThreads) k_compact_scan(SimDev* __restrict__ S, int nblocks)
{
    __shared__ int wsum[kScanThreads / 64];
    __shared__ int carry[2];
    if (threadIdx.x < 2) carry[threadIdx.x] = 0;
    __syncthreads();
    for (int base = 0; base < nblocks; base += kScanThreads) {
        const int b = base + threadIdx.x;
        const int a = b < nblocks ? S->sort_part[2 * b] : 0, u = b < nblocks ? S->sort_part[2 * b + 1] : 0;
        int sa, su;
        const int pa = block_scan(a, wsum, &sa) - a + carry[0];
        const int pu = block_scan(u, wsum, &su) - u + carry[1];
        if (b < nblocks) {
            S->sort_part[2 * b] = pa;
            S->sort_part[2 * b + 1] = pu;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            carry[0] += sa;
            carry[1] += su;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int ta = carry[0], tu = carry[1];
        const bool fits = ta <= S->max_slots && tu <= S->max_units;
        S->sort_part[kPartCopies * kRadix - 1] = fits ? 1 : 0;
        *S->n_active = fits ? ta : 0;
        *S->n_units = fits ? tu : 0;
        if (!fits) atomicAdd(S->over_count, 1ull << 40);
    }
}

// A list of one round (small grids): the three steps in one block and one launch.
__global__ void __launch_bounds__(kScanThreads) k_compact_one(SimDev* __restrict__ S)
{
    __shared__ int wsum[kScanThreads / 64];
    const CompactGeom G(S);
    const int U = S->unit_cap;
    int c[kCompactK], tt[kCompactK];
    int ra = 0, ru = 0;
    G.tiles_of(S, threadIdx.x * kCompactK, tt);
#pragma unroll
    for (int j = 0; j < kCompactK; ++j) {
        c[j] = tt[j] >= 0 ? compact_count(S, tt[j]) : 0;
        ra += c[j] > 0 ? 1 : 0;
        ru += compact_units(S, c[j]);
    }
    int ta, tu;
    int pa = block_scan(ra, wsum, &ta) - ra;
    int pu = block_scan(ru, wsum, &tu) - ru;
    const bool fits = ta <= S->max_slots && tu <= S->max_units;
#pragma unroll
    for (int j = 0; j < kCompactK; ++j) {
        const int t = tt[j];
        if (t < 0) continue;
        if (c[j] > 0 && fits) {
            const int k = compact_units(S, c[j]);
            S->active[pa] = t;
            S->tile_slot[t] = pu;
            S->tile_nslot[t] = k;
            for (int q = 0; q < k; ++q) {
                int* u = S->units + 3 * (pu + q);
                u[0] = t;
                u[1] = U > 0 ? q * U : 0;
                u[2] = U > 0 ? min(c[j], (q + 1) * U) : c[j];
            }
            ++pa;
            pu += k;
        } else {
            S->tile_slot[t] = -1;
            S->tile_nslot[t] = 0;
        }
    }
    if (threadIdx.x == 0) {
        *S->n_active = fits ? ta : 0;
        *S->n_units = fits ? tu : 0;
        if (!fits) atomicAdd(S->over_count, 1ull << 40);
    }
}

__global__ void __launch_bounds__(kScanThreads) k_compact_place(SimDev* __restrict__ S)
{
    __shared__ int wsum[kScanThreads / 64];
    const CompactGeom G(S);
    const int U = S->unit_cap;
    const bool fits = S->sort_part[kPartCopies * kRadix - 1] != 0;
    int oa = S->sort_part[2 * blockIdx.x], ou = S->sort_part[2 * blockIdx.x + 1];  // the blocks before
    const int r0 = blockIdx.x * G.rpb, r1 = min(G.rounds, r0 + G.rpb);
    for (int round = r0; round < r1; ++round) {
        int c[kCompactK], tt[kCompactK];
        int ra = 0, ru = 0;
        G.tiles_of(S, round * kCompactK * kScanThreads + threadIdx.x * kCompactK, tt);
#pragma unroll
        for (int j = 0; j < kCompactK; ++j) {
            c[j] = tt[j] >= 0 ? compact_count(S, tt[j]) : 0;
            ra += c[j] > 0 ? 1 : 0;
            ru += compact_units(S, c[j]);
        }
        int sa, su;
        int pa = block_scan(ra, wsum, &sa) - ra + oa;
        int pu = block_scan(ru, wsum, &su) - ru + ou;
#pragma unroll
        for (int j = 0; j < kCompactK; ++j) {
            const int t = tt[j];
            if (t < 0) continue;
            if (c[j] > 0 && fits) {
                const int k = compact_units(S, c[j]);
                S->active[pa] = t;
                S->tile_slot[t] = pu;
                S->tile_nslot[t] = k;
                for (int q = 0; q < k; ++q) {
                    int* u = S->units + 3 * (pu + q);
                    u[0] = t;
                    u[1] = U > 0 ? q * U : 0;
                    u[2] = U > 0 ? min(c[j], (q + 1) * U) : c[j];
                }
                ++pa;
                pu += k;
            } else {
                S->tile_slot[t] = -1;
                S->tile_nslot[t] = 0;
            }
        }
        oa += sa;
        ou += su;
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
            const int fuse = nb <= kFuseBlocks ? 1 : 0;
            hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortBlock), 0, st, dS, s, p, ipb, fuse);
            if (!fuse) hipLaunchKernelGGL(k_radix_rowsum, dim3(kRadix), dim3(kScanThreads), 0, st, dS, s, ipb);
            hipLaunchKernelGGL(k_radix_rowscan, dim3(kRadix), dim3(kScanThreads), 0, st, dS, s, ipb);
            if (ipb >= 4 * kSortBlock)
                hipLaunchKernelGGL(k_radix_scatter<4>, dim3(nb), dim3(kSortBlock), 0, st, dS, s, p, ipb);
            else
                hipLaunchKernelGGL(k_radix_scatter<1>, dim3(nb), dim3(kSortBlock), 0, st, dS, s, p, ipb);
        }
        hipLaunchKernelGGL(k_permute, dim3(g > 0 ? g : 1), dim3(256), 0, st, dS, s, passes, elem);
    }
    return hipGetLastError();
}

hipError_t enqueue_keys_only(SimDev* dS, int s, int n, hipStream_t st)
{
    const int g = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_keys, dim3(g > 0 ? g : 1), dim3(256), 0, st, dS, s);
    return hipGetLastError();
}

hipError_t enqueue_ranges(SimDev* dS, int s, int ntiles, int passes, bool swap, hipStream_t st)
{
    const int g = (ntiles + 1 + 255) / 256;
    hipLaunchKernelGGL(k_tile_ranges, dim3(g), dim3(256), 0, st, dS, s, passes, swap ? 1 : 0);
    return hipGetLastError();
}

hipError_t enqueue_compact(SimDev* dS, const SimDev& h, hipStream_t st)
{
    // the padded ranks of the list (as CompactGeom counts them) and its rounds, over at most
    // kCompactBlocks blocks
    long long nt = 1;
    for (int a = 0; a < 3; ++a) {
        const int b = a < h.dims ? kUnitBlock : 1;
        nt *= (long long)((h.ntile[a] + b - 1) / b) * b;
    }
    const long long rounds = (nt + kCompactK * kScanThreads - 1) / (kCompactK * kScanThreads);
    if (rounds <= 1) {
        hipLaunchKernelGGL(k_compact_one, dim3(1), dim3(kScanThreads), 0, st, dS);
        return hipGetLastError();
    }
    const int nb = (int)(rounds < kCompactBlocks ? rounds : kCompactBlocks);
    hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(kScanThreads), 0, st, dS);
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(kScanThreads), 0, st, dS, nb);
    hipLaunchKernelGGL(k_compact_place, dim3(nb), dim3(kScanThreads), 0, st, dS);
    return hipGetLastError();
}

}  // namespace pic

namespace pic {

// ---- untyped helpers ---------------------------------------------------------------------------
// even words get lo, odd words hi (a 64-bit pattern; lo == hi for a 32-bit one)
__global__ void k_fill(unsigned* __restrict__ p, long long nwords, unsigned lo, unsigned hi)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nwords; i += (long long)gridDim.x * blockDim.x)
        p[i] = (i & 1) ? hi : lo;
}

hipError_t enqueue_fill_pattern(void* p, size_t bytes, unsigned lo, unsigned hi, hipStream_t st)
{
    const long long nw = (long long)(bytes / 4);
    if (nw <= 0) return hipSuccess;
    long long g = (nw + 255) / 256;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(256), 0, st, reinterpret_cast<unsigned*>(p), nw, lo, hi);
    return hipGetLastError();
}

hipError_t enqueue_fill(void* p, size_t bytes, hipStream_t st) { return enqueue_fill_pattern(p, bytes, 0u, 0u, st); }

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

// ---- measurement helper: a structure-of-arrays streaming copy of known size ----
struct SoaPtrs {
    const float* src[PIC_MEASURE_MAX_ARRAYS];
    float* dst[PIC_MEASURE_MAX_ARRAYS];
};

__global__ void __launch_bounds__(256) k_measure_soa_copy(SoaPtrs p, int narrays, long long n)
{
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        float v[PIC_MEASURE_MAX_ARRAYS];
#pragma unroll
        for (int k = 0; k < PIC_MEASURE_MAX_ARRAYS; ++k)
            if (k < narrays) v[k] = p.src[k][i];
#pragma unroll
        for (int k = 0; k < PIC_MEASURE_MAX_ARRAYS; ++k)
            if (k < narrays) p.dst[k][i] = v[k];
    }
}

}  // namespace pic

extern "C" int pic_measure_soa_copy(const float* const* src, float* const* dst, int narrays, long long n,
                                    void* hip_stream)
{
    if (!src || !dst || narrays < 1 || narrays > PIC_MEASURE_MAX_ARRAYS || n < 0) return PIC_EINVAL;
    pic::SoaPtrs p{};
    for (int k = 0; k < narrays; ++k) {
        if (!src[k] || !dst[k]) return PIC_EINVAL;
        p.src[k] = src[k];
        p.dst[k] = dst[k];
    }
    if (n == 0) return PIC_OK;
    const long long blocks = (n + 255) / 256;
    const int grid = (int)(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(pic::k_measure_soa_copy, dim3(grid), dim3(256), 0, reinterpret_cast<hipStream_t>(hip_stream),
                       p, narrays, n);
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_EDEVICE;
}

// pic_sort.h -- enqueue functions of the cell sort (pic_sort.hip).
#pragma once
#include "pic_internal.h"

namespace pic {

// Keys per radix-sort block: 4096, doubled until at most 2048 blocks cover n keys (the digit
// histogram holds 256 counts per block), and for small sorts halved down to 1024 (one key per
// thread) while fewer than 512 blocks would cover them, so that the blocks fill the 256 CUs.
inline int sort_ipb(long long n)
{
    long long ipb = 4096;
    while ((n + ipb - 1) / ipb > 2048) ipb *= 2;
    while (ipb > 1024 && (n + ipb - 1) / ipb < 512) ipb /= 2;
    return (int)ipb;
}

// Stable radix sort of species s by cell key (passes of 8 bits) and permutation of its arrays
// into the alternates.  elem = 4 (FP32 form) or 8 (FP64 form).  enqueue_ranges with swap = true
// must follow: it swaps the arrays with their alternates.
hipError_t enqueue_sort(SimDev* dS, int s, int n, int passes, int elem, hipStream_t st);
// Per-tile particle ranges of species s from its sorted keys; after a sort of s, swap = true.
hipError_t enqueue_ranges(SimDev* dS, int s, int ntiles, int passes, bool swap, hipStream_t st);
// Keys of species s into its key buffer (diagnostics).
hipError_t enqueue_keys_only(SimDev* dS, int s, int n, hipStream_t st);
// Active tile list and slots.
hipError_t enqueue_compact(SimDev* dS, const SimDev& h, hipStream_t st);

}  // namespace pic

/* pic_measure.h -- measurement helper of libpic (not part of the method).
 *
 * A streaming copy of known size with the particle kernel's access pattern:
 * structure-of-arrays float arrays, each lane loading and storing one 4-byte
 * element of every array.  Profilers count HBM bytes per dispatch through
 * hardware counters whose units depend on the request sizes a kernel issues;
 * dividing this copy's exact byte count by what a counter reports for it gives
 * the factor to apply to the particle kernel in the same run. */
#ifndef PIC_MEASURE_H
#define PIC_MEASURE_H

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_MEASURE_MAX_ARRAYS 16

/* dst[k][i] = src[k][i] for k < narrays, i < n, enqueued on hip_stream (the
 * host does not wait).  src and dst are host arrays of narrays device
 * pointers to n floats each (not overlapping).  Bytes moved: 4 n narrays read
 * and as many written.  Errors: PIC_EINVAL (narrays outside
 * [1, PIC_MEASURE_MAX_ARRAYS], n < 0, a null pointer), PIC_EDEVICE. */
int pic_measure_soa_copy(const float* const* src, float* const* dst, int narrays, long long n,
                         void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif

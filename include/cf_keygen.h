/*
 * cf_keygen.h -- device-side synthetic key generator shipped in libcf.so.
 *
 * Not part of the filter's method: it fills device buffers with the seeded
 * uniform 64-bit keys the benchmarks and large tests feed to the filter, so
 * that inputs of several GiB need not cross PCIe.  Key number c of stream
 * `seed` is output c of SplitMix64 (Steele, Lea and Flood 2014) started at
 * state `seed`:  z = seed + (c + 1) * 0x9e3779b97f4a7c15, followed by the
 * SplitMix64 output mix.  Counter -> key is a bijection, so distinct
 * counters give distinct keys.
 */
#ifndef CF_KEYGEN_H
#define CF_KEYGEN_H

#include <stdint.h>

#include "cf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* d_out[i] = key(seed, start + i) for 0 <= i < n.  d_out: device uint64[n],
 * 8-byte aligned, owned by the caller.  Stream-ordered; CF_EINVAL for a NULL
 * buffer with n > 0, CF_EDEVICE on a launch error. */
cf_status cf_keygen(uint64_t *d_out, uint64_t n, uint64_t seed, uint64_t start,
                    void *stream);

/* d_out[i] = key(seed, counters[i]): keys for an arbitrary device array of
 * counters (uint64[n]).  Same error behaviour as cf_keygen. */
cf_status cf_keygen_at(uint64_t *d_out, const uint64_t *d_counters, uint64_t n,
                       uint64_t seed, void *stream);

/* Memory-system probe for the benchmark's roofline, not part of the method:
 * n_reads independent reads, one per thread, each of `width` bytes (8 or 16)
 * at the start of line L_i = (key(seed, i) mod n_lines) of the device buffer
 * d_buf, which holds n_lines lines of line_bytes bytes.  This is the access
 * pattern of a bucket probe into a large table, without the filter's work,
 * so its rate is the ceiling a probe-bound kernel can reach.  n_lines and
 * line_bytes are powers of two, line_bytes >= width; d_buf is 16-byte
 * aligned and caller-owned.  Each thread sums what it loaded and adds 1 to
 * *d_sink (a device uint64, 8-byte aligned) only when that sum equals a fixed
 * constant, so the compiler keeps every load and the probe writes almost
 * nothing.  Stream-ordered; CF_EINVAL for bad arguments, CF_EDEVICE on a
 * launch error. */
cf_status cf_probe_lines(const void *d_buf, uint64_t n_lines, uint32_t line_bytes,
                         uint32_t width, uint64_t n_reads, uint64_t seed, uint64_t *d_sink,
                         void *stream);

/* Memory-system probe, the atomic counterpart of cf_probe_lines: n_ops
 * device-scope 64-bit compare-and-swaps, one per thread, on the first 8-byte
 * word of line L_i = (key(seed, i) mod n_lines) of d_buf (n_lines lines of
 * line_bytes bytes), the access of a bucket update (Alg. 1 and 3 claim and
 * clear slots with such a CAS).  read_first = 1 loads the word first and
 * swaps it for a changed value, as a bucket update does; read_first = 0
 * issues the CAS without a read, expecting 0.  The probe CHANGES the words
 * it hits: d_buf is caller-owned scratch, 8-byte aligned.  n_lines and
 * line_bytes are powers of two, line_bytes >= 8; *d_sink (8-byte aligned)
 * takes 1 only when a thread's sum of returned values equals a fixed
 * constant.  Stream-ordered; CF_EINVAL for bad arguments, CF_EDEVICE on a
 * launch error. */
cf_status cf_probe_atomics(void *d_buf, uint64_t n_lines, uint32_t line_bytes,
                           uint32_t read_first, uint64_t n_ops, uint64_t seed, uint64_t *d_sink,
                           void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CF_KEYGEN_H */

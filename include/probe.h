/* probe.h -- C ABI of the HBM bandwidth probe: hand-written streaming
 * kernels that measure the practical memory ceiling the phase-field LBM
 * kernels are compared with, beside MI355X's published 8 TB/s.  It is
 * measurement infrastructure, not part of the method.
 *
 * pb_stream(kind, src, dst, n, q, reps, stream, ms_out): `reps` timed passes
 * after one untimed pass, on `stream` (hipStream_t, NULL = default), timed
 * with HIP events on that stream; *ms_out receives the mean milliseconds per
 * pass.  Synchronises the stream.  Buffers are caller-owned device memory of
 * n floats (n a positive multiple of 4, below 2^33):
 *   kind 0  copy src -> dst, 16 bytes per lane, one block of 256 lanes per
 *           4 KiB (bytes moved per pass: 8 n);
 *   kind 1  the same copy with non-temporal loads and stores (8 n);
 *   kind 2  read src, 16 bytes per lane, keeping the sum in registers
 *           (4 n; dst receives one float per block only if a sum equals a
 *           sentinel value, i.e. in practice never, and must hold n / 1024
 *           floats);
 *   kind 3  in place on src, viewed as q arrays of n / q floats (q = 19 or
 *           38, n a multiple of q), blocks of 512 lanes as the fused step's
 *           256 x 2 tiles: every lane reads its element of all q arrays, then stores them back in reverse array order, the
 *           access pattern of the fused step at its even parity (8 n;
 *           src's contents are permuted; dst unused);
 *   kind 4  as kind 3 on q arrays of 2 n / q 16-bit values, one value per
 *           lane (2-byte accesses, 8 n);
 *   kind 5  as kind 4 with two adjacent values per lane (4-byte accesses,
 *           8 n);
 *   kind 6  src viewed as q arrays of n / q floats, read; their sum per
 *           element written to dst (n / q floats), 512-lane blocks: the
 *           phase-field pass's pattern (4 n + 4 n / q).
 * Returns 0, or a negative code with pb_last_error() describing it (per
 * thread): -1 bad argument, -3 device error. */
#pragma once
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

int pb_stream(int kind, void* src, void* dst, size_t n, int q, int reps, void* stream, double* ms_out);
const char* pb_last_error(void);

#ifdef __cplusplus
}
#endif

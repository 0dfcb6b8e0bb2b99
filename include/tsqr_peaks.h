/*
 * tsqr_peaks.h -- C ABI of libtsqr_peaks: the machine ceilings that the
 * roofline fractions of the TSQR kernels are quoted against, measured on the
 * part itself rather than taken from the datasheet.  Not part of the
 * factorisation; the TSQR library does not link it.
 *
 * The byte and flop model of the method (A read, reflectors written and read,
 * Q written: Sec. 4.1; the flop count of Sec. 4.2) makes every step
 * HBM-bound on this part; its ceiling is what a plain streaming copy reaches.
 * The dense contractions run on the FP64 matrix cores and the reflector
 * arithmetic on the FP64 vector ALU, so both FP64 rates are measured too.
 *
 * Conventions:
 *   - Every pointer is a DEVICE pointer owned by the caller; calls are
 *     asynchronous on `stream` (a hipStream_t, NULL = the default stream) and
 *     return once the kernel is enqueued.  The caller times them with events
 *     on that stream.
 *   - grid <= 0 picks the default launch: for the streams, one pass over the
 *     buffer (workgroups of 256 threads, each taking one chunk of 256 x 16
 *     bytes for the copy and 4 x 256 x 16 bytes for the read, at most
 *     1 << 20 workgroups, which then loop over further chunks); for the loops,
 *     8 workgroups of 256 threads per compute unit.  Otherwise
 *     1 <= grid <= 1 << 20.
 *   - Status: 0 = success, -i = argument i (1-based) invalid, 1 = HIP launch
 *     error.
 */
#ifndef TSQR_PEAKS_H
#define TSQR_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dst[0 .. bytes) = src[0 .. bytes) with 16-byte loads and stores.  Both
 * pointers 16-byte aligned, bytes a positive multiple of 16, the buffers
 * disjoint.  HBM traffic: 2 * bytes. */
int tsqr_peak_copy(const void* src, void* dst, int64_t bytes, int grid, void* stream);

/* Streaming read: partial[g] = sum of the FP64 values in the part of
 * src[0 .. bytes) that workgroup g visits (16-byte loads, grid-stride order),
 * so sum(partial) = sum of all bytes / 8 doubles.  src 16-byte aligned, bytes
 * a positive multiple of 16; partial holds `grid` doubles (the default grid's
 * size is returned by tsqr_peak_grid(1, bytes)).  HBM traffic: bytes. */
int tsqr_peak_read(const void* src, int64_t bytes, double* partial, int grid, void* stream);

/* Copy of the column-major m x n matrix src (leading dimension lds) into dst
 * (ldd) in the access pattern of the TSQR Q kernel, without its arithmetic:
 * one wavefront per leaf of leaf_rows rows (floor(m / leaf_rows) leaves, at
 * least one, the last taking the remaining rows), its tiles of tile_rows rows
 * walked from the last to the first, 16 rows at a time, lane 16 g + r moving
 * row r of those in columns 4 k + g.  Requirements: lds, ldd >= m >= 1,
 * 1 <= n <= 64, tile_rows a positive multiple of 16, leaf_rows a multiple of
 * tile_rows, the two matrices disjoint (-3 otherwise).  The ceiling of that
 * access pattern at that concurrency.  HBM traffic: 16 m n bytes. */
int tsqr_peak_copy_leaf(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t m, int n,
                        int64_t leaf_rows, int tile_rows, void* stream);

/* FP64 FMA loop on the vector ALU: every thread runs `iters` rounds of eight
 * independent chains x <- fma(x, c, d) started at x = 0 .. 7 and writes the
 * sum of the eight results to out[thread] (grid * 256 doubles).  With c = 1,
 * d = 1 the exact result is 28 + 8 * iters.  Flops: 16 * iters per thread. */
int tsqr_peak_fma(double* out, int grid, int iters, double c, double d, void* stream);

/* FP64 matrix-core loop: every wavefront runs `iters` rounds of 16 steps on
 * each of four independent 16x16x4 FP64 MFMA chains D <- A B + D, every entry
 * of A equal to a and of B equal to b, D starting at zero; each thread writes
 * the sum of its 16 accumulator entries to out[thread] (grid * 256 doubles).
 * The exact result is 1024 * a * b * iters when that is exactly
 * representable.  Flops: 131072 * iters per wavefront. */
int tsqr_peak_mfma(double* out, int grid, int iters, double a, double b, void* stream);

/* The grid a call with grid <= 0 launches on the current device: kind 0 =
 * tsqr_peak_copy of `bytes` bytes, 1 = tsqr_peak_read of `bytes` bytes, 2 = the
 * FMA and MFMA loops (bytes unused).  -1 for a bad kind or a HIP error. */
int tsqr_peak_grid(int kind, int64_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* TSQR_PEAKS_H */

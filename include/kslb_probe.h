/*
 * kslb_probe.h -- measurement kernels of libkslb_probe (gfx950): the device
 * peaks the solver's kernels are compared with.  Not part of the method;
 * they compute nothing of the lattice Boltzmann scheme.
 *
 * Every function enqueues work on the caller's stream (a hipStream_t; NULL =
 * the null stream) and returns a hipError_t as int (0 = success); buffers
 * belong to the caller.
 */
#ifndef KSLB_PROBE_H
#define KSLB_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* STREAM-style copy: dst[i] = src[i] for bytes (a multiple of 16) bytes of
 * 16-byte aligned device memory, 16 bytes per lane per access, four loads
 * per lane in flight before its stores (streaming stores), one workgroup per
 * 16 KiB.  Moves 2 * bytes through HBM when the buffers exceed the
 * last-level caches.                                                      */
int kslb_probe_copy(void* dst, const void* src, size_t bytes, void* stream);

/* LDS read bandwidth: blocks workgroups of 256 lanes, each filling 32 KiB of
 * LDS and then reading it iters times with 16-byte loads whose addresses
 * are consecutive across a wave (conflict-free), folding the values into a
 * result no compiler can drop.  out (device, 4 * blocks 64-bit words):
 * per workgroup its LDS bytes read, the shader clocks of its read loop
 * (s_memtime), the constant 100 MHz clock ticks of the same interval
 * (s_memrealtime) and the folded value.                                    */
int kslb_probe_lds(uint64_t* out, int blocks, int iters, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KSLB_PROBE_H */

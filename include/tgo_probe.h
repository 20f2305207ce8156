/*
 * tgo_probe -- calibration library (libtgo_probe.so), not part of the tgo
 * product ABI.  It measures the device, not the model: the benchmark runs it
 * under a counter profiler to obtain the 32-bit VALU issue rate that the
 * ALU-bound roofline of the enumeration kernels is priced against.
 */
#ifndef TGO_PROBE_H
#define TGO_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Integer issue probe: `blocks` (1..2^20) blocks of 256 threads, each thread
 * running eight independent chains of 32-bit shift-and-add for iters (1..2^20)
 * x 16 steps (2 VALU instructions per step and chain, no memory traffic).
 * d_sink: a device buffer of at least 4 bytes (written only in a case that
 * does not occur, which keeps the chains from being optimised away).  Enqueued
 * on `stream` (a hipStream_t).  Returns 0, -1 for a bad argument, -4 for a HIP
 * launch error. */
int tgo_probe_valu(int blocks, int iters, void *d_sink, void *stream);

#ifdef __cplusplus
}
#endif

#endif

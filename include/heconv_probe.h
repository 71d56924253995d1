/*
 * heconv_probe.h -- measured integer-VALU ceilings for the library's kernels
 * (measurement only; no part of the homomorphic computation).
 *
 * The transforms and the MAC are bound by the GPU's integer vector issue
 * rate or by HBM.  he_probe_valu measures the first: one instruction, or one
 * kernel's arithmetic on operands held in registers (no memory traffic in
 * the loop), over a grid that fills every compute unit, timed with HIP
 * events.  The kernel-mix probes run the same device functions as the
 * kernels, so their rates are the ceilings of those kernels' own
 * instruction mixes.
 */
#ifndef HECONV_PROBE_H
#define HECONV_PROBE_H

#include <stdint.h>

#include "heconv.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HE_PROBE_MAD_U64_U32 = 0, /* v_mad_u64_u32, lane operations/s */
  HE_PROBE_MUL_HI_U32 = 1,  /* v_mul_hi_u32, lane operations/s */
  HE_PROBE_MUL_LO_U32 = 2,  /* v_mul_lo_u32, lane operations/s */
  HE_PROBE_ADD_U32 = 3,     /* v_add_u32 (full-rate reference), lane operations/s */
  HE_PROBE_MAC_MIX = 4,     /* the batch MAC's 6x4-tile channel-block step and carry, products/s */
  HE_PROBE_INTT_MIX = 5,    /* the inverse transform's butterfly, butterflies/s */
  HE_PROBE_NTT_MIX = 6      /* the forward transform's butterfly, butterflies/s */
};

/* Run probe `which` (iters loop trips per thread, `blocks` workgroups of 256
 * threads) twice on `stream`, the second launch timed; *ops_per_s receives
 * the rate in the probe's unit.  The kernel-mix probes use the first prime
 * of ctx.  d_work: 64 + 256*blocks device words; the first 64 hold any
 * values (operand seeds), the rest is overwritten.  Synchronises `stream`.
 * HE_EINVAL for an unknown probe, zero counts or null pointers. */
he_status he_probe_valu(const he_ctx* ctx, uint32_t which, uint32_t iters, uint32_t blocks, uint64_t* d_work,
                        double* ops_per_s, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HECONV_PROBE_H */

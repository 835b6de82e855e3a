/* dqj_measure.h -- measurement helpers of the dqj library (libdqj.so), beside the
 * rendering ABI of dqj.h. These calls do no rendering; they report what the device
 * sustains, so that throughput can be set against the clock the chip actually ran at.
 *
 * Calls return a dqj_status; the text of the last failure is dqj_last_error(). */
#ifndef DQJ_MEASURE_H
#define DQJ_MEASURE_H

#include <stdint.h>

#include "dqj.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Engine (shader) clock that device `device` sustains under an FP32 FMA load, in MHz.
 * Purpose: the FP32 vector peak is 256 flop/clk per compute unit times the engine clock;
 * under a long VALU load the clock settles below the nominal one, and this call measures
 * it, for a peak at the clock actually run. (Measurement support: the paper gives no
 * hardware figures.)
 *
 * How: one launch fills every compute unit with 8 waves per SIMD, each running chains of
 * dependent FMAs for about `seconds` of wall time. Each wave reads the shader clock
 * counter and the constant-rate wall clock counter before and after its loop; the result
 * is the sum of the shader clock deltas over the sum of the wall clock deltas, times the
 * wall clock's rate (hipDeviceAttributeWallClockRate).
 *
 * Arguments: `device` is a HIP device index; `seconds` in (0, 10] is the length of the
 * load (a first short launch of about a millisecond sets the loop count, which is capped
 * at 3e7 rounds, about 10 s at the measured rate); `mhz` (host pointer, written on
 * success) receives the clock. The call allocates a small device buffer, launches on the
 * device's null stream, waits for the whole device (hipDeviceSynchronize) and frees the
 * buffer before it returns; it leaves the current device as it found it. Other work on the
 * device while it runs shares the load and lowers nothing but the accuracy.
 *
 * Errors: DQJ_E_INVALID for a NULL `mhz`, `seconds` out of range or no such device;
 * DQJ_E_UNSUPPORTED for a device that is not gfx950; DQJ_E_NOMEM or DQJ_E_DEVICE for
 * HIP failures. Nothing is written to `mhz` on failure. */
dqj_status dqj_measure_engine_clock(int32_t device, double seconds, double *mhz);

#ifdef __cplusplus
}
#endif
#endif

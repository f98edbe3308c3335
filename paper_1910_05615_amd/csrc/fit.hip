// Full RT-DetMCD fit orchestration (filled in below).
#include "driver.h"

extern "C" {
rtdetmcd_status rtdetmcd_fit(rtdetmcd_handle ctx, const void*, int32_t, int64_t, int32_t, int64_t,
                             int64_t, int32_t, const rtdetmcd_opts*, const rtdetmcd_out*) {
  if (ctx) ctx->err = "not implemented";
  return RTDETMCD_EUNSUPPORTED;
}
rtdetmcd_status rtdetmcd_fit_batched(rtdetmcd_handle ctx, int32_t, const rtdetmcd_dataset*,
                                     const rtdetmcd_opts*, rtdetmcd_status*) {
  if (ctx) ctx->err = "not implemented";
  return RTDETMCD_EUNSUPPORTED;
}
}

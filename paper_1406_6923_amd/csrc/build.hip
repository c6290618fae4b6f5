// Stage 1 of Algorithm 1 on the device (ROM construction) -- entry point.
#include "sfm_internal.h"

extern "C" sfm_status sfm_build_roms(sfm_ctx c, const float* vel_dev, int32_t nsrc, const int32_t* src_ijk,
                                     int32_t nrec, const int32_t* rec_ijk, const float* u0_dev,
                                     const float* v0_dev, void* stream) {
  (void)vel_dev; (void)nsrc; (void)src_ijk; (void)nrec; (void)rec_ijk; (void)u0_dev; (void)v0_dev; (void)stream;
  if (!c) return SFM_EINVAL;
  return c->fail(SFM_EINVAL, "device ROM build is not available in this build");
}

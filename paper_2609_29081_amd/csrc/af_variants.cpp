// af_variants.cpp -- registry of the compiled variants of the 2D stage (one
// object file of af_stage2d.hip each; the list matches STAGE_VARIANTS in
// build.py) and the single-instance stage, which uses the default variant of
// its precision.
#include "af_internal.hpp"

namespace afi {

#define AF_DECLARE_VARIANT(name)                                                               \
  hipError_t name(const Geo&, const afd::Phys&, const Work&, const double*, const double*,    \
                  double*, const double*, double, StageCoef, hipStream_t, Timer*);            \
  hipError_t name##_batch(BatchInst*, int, int, const int*, int, hipStream_t, Timer*);        \
  hipError_t name##_dev(const Geo&, const afd::Phys&, BatchInst*, double*, int, hipStream_t); \
  int name##_nwg(const Geo&);                                                                 \
  int name##_tiles(const Geo&);

AF_DECLARE_VARIANT(stage2d_fp64_t7)
AF_DECLARE_VARIANT(stage2d_fp64_t5)
AF_DECLARE_VARIANT(stage2d_mixed_t10)
AF_DECLARE_VARIANT(stage2d_mixed_t7)
AF_DECLARE_VARIANT(stage2d_mixed_t14)

#define AF_VARIANT(name, mixed, ty) \
  {#name, mixed, ty, name, name##_batch, name##_tiles, name##_dev, name##_nwg}

const StageVariant kStageVariants[] = {
    AF_VARIANT(stage2d_fp64_t7, 0, 7),    AF_VARIANT(stage2d_fp64_t5, 0, 5),
    AF_VARIANT(stage2d_mixed_t14, 1, 14), AF_VARIANT(stage2d_mixed_t10, 1, 10),
    AF_VARIANT(stage2d_mixed_t7, 1, 7)};
const int kNumStageVariants = sizeof(kStageVariants) / sizeof(kStageVariants[0]);

const StageVariant* default_variant(int mixed) {
  for (int i = 0; i < kNumStageVariants; ++i)
    if (kStageVariants[i].mixed == (mixed ? 1 : 0)) return &kStageVariants[i];
  return &kStageVariants[0];
}

hipError_t stage2d(const Geo& g, const afd::Phys& ph, const Work& w, const double* Un,
                   const double* Uk, double* Uout, const double* dt_dev, double dt_host,
                   StageCoef sc, hipStream_t s, Timer* tm) {
  return default_variant(g.mixed)->single(g, ph, w, Un, Uk, Uout, dt_dev, dt_host, sc, s, tm);
}

}  // namespace afi

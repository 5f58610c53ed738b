// Multilevel layout (Sec. 2, Algorithms 1-3).
#include "vmo_internal.h"

namespace vmo {
void layout(Ctx&, const vmo_hypergraph*, const vmo_layout_params*, float*, hipStream_t) {
  throw Error(VMO_E_UNSUPPORTED, "layout not built yet");
}
void coarsen(Ctx&, const vmo_hypergraph*, uint64_t, uint64_t, int32_t, int32_t, int32_t*, int64_t*, int32_t*, float*,
             float*, int32_t*, int32_t*, hipStream_t) {
  throw Error(VMO_E_UNSUPPORTED, "layout not built yet");
}
void tree(Ctx&, const float*, const float*, int32_t, int32_t, int32_t*, int32_t*, float*, int32_t*, int32_t, int32_t*,
          hipStream_t) {
  throw Error(VMO_E_UNSUPPORTED, "layout not built yet");
}
void gradient(Ctx&, const vmo_hypergraph*, const float*, float, int32_t, float*, float*, int64_t*, hipStream_t) {
  throw Error(VMO_E_UNSUPPORTED, "layout not built yet");
}
void layout_steps(Ctx&, const vmo_hypergraph*, const vmo_layout_params*, float*, int32_t, int32_t, double*,
                  hipStream_t) {
  throw Error(VMO_E_UNSUPPORTED, "layout not built yet");
}
}  // namespace vmo

// Tuned 3-D kernels (filled in once the generic path is parity-green).
#include "sem_internal.h"

namespace sem {

bool fast3d_supported(int, int) { return false; }
int64_t fast3d_face_values(const ProbDev&) { return 0; }
hipError_t launch_fast3d(const ProbDev&, int, const void*, const void*, void*, void*, const Epi&, Coef, const void*,
                         hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace sem

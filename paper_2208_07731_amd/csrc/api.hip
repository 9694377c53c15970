// Version and status strings of libisdf.
#include "common.h"

extern "C" const char* isdf_version(void) { return "isdf-mi355x 0.1.0 (gfx950)"; }

extern "C" const char* isdf_strerror(int status) {
  switch (status) {
    case ISDF_OK: return "ok";
    case ISDF_E_ARG: return "invalid argument";
    case ISDF_E_WORKSPACE: return "workspace too small";
    case ISDF_E_HIP: return "HIP runtime error while enqueueing";
    case ISDF_E_UNSUPPORTED: return "unsupported combination of arguments";
    case ISDF_E_SCRATCH: return "request exceeds the static scratch of the allocation-free entry point";
    case ISDF_E_NOT_PD: return "C C^H is not positive definite";
    case ISDF_E_NONFINITE: return "non-finite value in the input";
    case ISDF_W_EMPTY_CLUSTER: return "a K-means cluster has no member";
    case ISDF_E_BAD_IDX: return "interpolation index out of range or repeated";
    default: return "unknown status";
  }
}

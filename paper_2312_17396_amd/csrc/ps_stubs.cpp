// Entry points declared in ps.h that are not implemented yet.
#include "ps_internal.h"

extern "C" {

ps_status ps_workspace_size_backward(ps_dtype, int, int64_t, int, int, int, int, size_t*) {
  return PS_ERR_UNSUPPORTED;
}
ps_status ps_expm_backward(ps_dtype, int, int64_t, const void*, int64_t, int64_t, const void*, int64_t, int64_t,
                           const double*, int, int, int, void*, int64_t, int64_t, int, const ps_opts*, void*, size_t,
                           void*) {
  return PS_ERR_UNSUPPORTED;
}

}  // extern "C"

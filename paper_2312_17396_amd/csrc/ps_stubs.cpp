// Entry points declared in ps.h that are not implemented yet.
#include "ps_internal.h"

extern "C" {

ps_status ps_workspace_size_batched(ps_dtype, int, const int32_t*, int, const int32_t*, size_t*) {
  return PS_ERR_UNSUPPORTED;
}
ps_status ps_expm_batched(ps_dtype, int, const int32_t*, const void* const*, const int64_t*, const double*, int,
                          const int32_t*, const int32_t*, void* const*, const int64_t*, const ps_opts*, int32_t*,
                          void*, size_t, void*) {
  return PS_ERR_UNSUPPORTED;
}
ps_status ps_batched_prepare(ps_dtype, int, const int32_t*, const void* const*, const int64_t*, const double*, int,
                             const int32_t*, const int32_t*, void* const*, const int64_t*, const ps_opts*, void*,
                             size_t, void*, ps_batched_handle*) {
  return PS_ERR_UNSUPPORTED;
}
ps_status ps_batched_launch(ps_batched_handle, void*) { return PS_ERR_UNSUPPORTED; }
ps_status ps_batched_destroy(ps_batched_handle) { return PS_ERR_UNSUPPORTED; }
ps_status ps_workspace_size_backward(ps_dtype, int, int64_t, int, int, int, int, size_t*) {
  return PS_ERR_UNSUPPORTED;
}
ps_status ps_expm_backward(ps_dtype, int, int64_t, const void*, int64_t, int64_t, const void*, int64_t, int64_t,
                           const double*, int, int, int, void*, int64_t, int64_t, int, const ps_opts*, void*, size_t,
                           void*) {
  return PS_ERR_UNSUPPORTED;
}

}  // extern "C"

#include "internal.hpp"
namespace malbec {
int launch_integrate_f32k(const malbec_run &, const StTable &, const int32_t *, int64_t, double *,
                          int32_t *, int32_t *, hipStream_t)
{ return fail(MALBEC_ENOTSUP, "F32_KAHAN not built yet"); }
int launch_camera(const malbec_camera &, double, double, int32_t *, int32_t *, double *, double *,
                  void *, hipStream_t)
{ return fail(MALBEC_ENOTSUP, "camera not built yet"); }
}

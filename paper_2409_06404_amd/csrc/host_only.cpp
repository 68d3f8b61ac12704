// Launchers of a host-only build of the library (api.cpp and mech.cpp without kernels.hip):
// every launcher reports that no device code is present.  This build loads mechanisms with
// device -1 and validates every call, so that the host code can be compiled and run with the
// address and undefined-behaviour sanitizers on a machine without a GPU; it never computes.
#include "crf_internal.h"

namespace crf {

hipError_t launch_thermo(const DevMech &, int64_t, const double *, const double *, int64_t, const double *,
                         int64_t, double *, double *, double *, double *, double *, double *, double *,
                         double *, hipStream_t) {
    return hipErrorNoBinaryForGpu;
}
hipError_t launch_wdot(const DevMech &, int, int64_t, const double *, const double *, int64_t, const double *,
                       int64_t, double *, double *, double *, double *, hipStream_t) {
    return hipErrorNoBinaryForGpu;
}
hipError_t launch_transport(const DevMech &, int, int64_t, const double *, const double *, int64_t,
                            const double *, int64_t, double *, double *, double *, hipStream_t) {
    return hipErrorNoBinaryForGpu;
}
hipError_t launch_vjp(const DevMech &, int, int64_t, const double *, const double *, int64_t, const double *,
                      int64_t, const double *, const double *, double *, double *, const double *, hipStream_t) {
    return hipErrorNoBinaryForGpu;
}
hipError_t launch_jvp(const DevMech &, int, int64_t, const double *, const double *, int64_t, const double *,
                      int64_t, const double *, const double *, double *, double *, double *, hipStream_t) {
    return hipErrorNoBinaryForGpu;
}
hipError_t launch_source(const DevMech &, int, int64_t, const double *, const double *, int64_t, const double *,
                         int64_t, double, double *, double *, double *, double *, hipStream_t) {
    return hipErrorNoBinaryForGpu;
}
hipError_t launch_reactor(const DevMech &, int, int64_t, double *, const double *, int64_t, double *, int64_t,
                          double, int, void *, hipStream_t) {
    return hipErrorNoBinaryForGpu;
}
hipError_t launch_reactor_static(const DevMech &, int, int64_t, double *, const double *, int64_t, double *,
                                 int64_t, double, int, hipStream_t) {
    return hipErrorNoBinaryForGpu;
}
hipError_t launch_peak(int, int64_t, int, double *, hipStream_t) { return hipErrorNoBinaryForGpu; }
hipError_t launch_jac(const DevMech &, int, int64_t, const double *, const double *, int64_t, const double *,
                      int64_t, void *, double *, hipStream_t) {
    return hipErrorNoBinaryForGpu;
}

}  // namespace crf

// float2 instantiation of the register-tiled pass kernels.
#include "pass2.hpp"

template cfh_status cfh::launch_pass2<float2>(uint64_t, hipStream_t, float2 *, const double2 *,
                                             const cfh::PassArgs2 &, int, double2 *, unsigned);
template cfh_status cfh::launch_adj2<float2>(uint64_t, hipStream_t, float2 *, float2 *, const double2 *,
                                            const cfh::PassArgs2 &, bool, double *, unsigned, double *);
template cfh_status cfh::launch_ham2<float2>(uint64_t, hipStream_t, const float2 *, float2 *, const double2 *,
                                             const cfh::PassArgs2 &, int);

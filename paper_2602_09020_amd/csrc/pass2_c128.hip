// double2 instantiation of the register-tiled pass kernels.
#include "pass2.hpp"

template cfh_status cfh::launch_pass2<double2>(uint64_t, hipStream_t, double2 *, const double2 *,
                                             const cfh::PassArgs2 &, int, double2 *, unsigned);
template cfh_status cfh::launch_adj2<double2>(uint64_t, hipStream_t, double2 *, double2 *, const double2 *,
                                            const cfh::PassArgs2 &, bool, double *, unsigned, double *);
template cfh_status cfh::launch_ham2<double2>(uint64_t, hipStream_t, const double2 *, double2 *, const double2 *,
                                             const cfh::PassArgs2 &, int);

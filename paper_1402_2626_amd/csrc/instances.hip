// Instances of the kernel launchers of launch.hpp for one level and one kind,
// chosen at compile time: PE_LEVEL (a level code: 1, 2 or 4, or 8 | 1, 2, 4
// for real numbers) and PE_KIND (0 rows, 1 adjoint,
// 2 batch, 3 Gauss-Newton in one workgroup, 4 column-parallel least squares).
// The build compiles this file once per pair.
#define PE_LAUNCH_DEFINITIONS
#include "launch.hpp"

#if !defined(PE_LEVEL) || !defined(PE_KIND)
#error "compile with -DPE_LEVEL=<1|2|4> -DPE_KIND=<0..4>"
#endif

namespace pe {

#if PE_KIND == 0
template hipError_t launch_rows<PE_LEVEL>(const EvalShape&, int, const double*, const OutView&, int, hipStream_t);
template hipError_t launch_terms<PE_LEVEL>(const EvalShape&, int, const double*, const OutView&, hipStream_t);
#elif PE_KIND == 1
template hipError_t launch_adjoint<PE_LEVEL>(const EvalShape&, int, const double*, const double*, int, int, double*,
                                             double*, hipStream_t);
#elif PE_KIND == 2
template hipError_t launch_batch<PE_LEVEL>(const BatchShape&, int, const double*, const BatchOut&, int, hipStream_t);
#elif PE_KIND == 3
template hipError_t launch_mgs<PE_LEVEL>(int, int, int, double*, int64_t, double*, int64_t, double*, int64_t, double*,
                                         double*, hipStream_t);
template hipError_t launch_mgs_batch<PE_LEVEL>(int, int, int, const BatchNewtonDesc*, const int*, double*, double*,
                                               double*, double*, double*, hipStream_t);
template hipError_t launch_rhs_shift<PE_LEVEL>(double*, int64_t, int64_t, int64_t, int, int, int, const double*, double,
                                               double, hipStream_t);
#elif PE_KIND == 4
template hipError_t launch_lstsq<PE_LEVEL>(const LsLayout&, void*, const double*, int64_t, int64_t, int64_t, double*,
                                           int64_t, int, double*, double*, double*, hipStream_t);
#endif

}  // namespace pe

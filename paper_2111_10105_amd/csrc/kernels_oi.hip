// Dispatch of the orthogonal iterations (Algorithm 1) to the kernel class of
// a problem: T up to 32 or 64 frames, k up to 16 or 32 (the 16-column tile of
// the matrix-core products).  The kernels themselves are in oi_device.h,
// instantiated once per class in kernels_oi_t<T>k<k>.hip.
#include "dmc_internal.h"

namespace dmc {

void launch_oi_batch(hipStream_t st, int tmax, int kr, int precision, const OiArgs* args,
                     const int4* jobs, int njobs) {
  if (njobs <= 0) return;
  prof::begin(st, DMC_KERNEL_OI);
  if (tmax <= 32)
    kr <= 16 ? launch_oi_batch_t<32, 16>(st, precision, args, jobs, njobs)
             : launch_oi_batch_t<32, 32>(st, precision, args, jobs, njobs);
  else
    kr <= 16 ? launch_oi_batch_t<64, 16>(st, precision, args, jobs, njobs)
             : launch_oi_batch_t<64, 32>(st, precision, args, jobs, njobs);
  prof::end(st, DMC_KERNEL_OI);
}

void launch_oi(hipStream_t st, const OiArgs& a) {
  prof::begin(st, DMC_KERNEL_OI);
  const int kt = a.k <= 16 ? 16 : 32;
  if (a.T <= 32)
    kt == 16 ? launch_oi_t<32, 16>(st, a) : launch_oi_t<32, 32>(st, a);
  else
    kt == 16 ? launch_oi_t<64, 16>(st, a) : launch_oi_t<64, 32>(st, a);
  prof::end(st, DMC_KERNEL_OI);
}

}  // namespace dmc

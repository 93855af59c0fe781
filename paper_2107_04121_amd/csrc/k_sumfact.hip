// Sum-factorized hexahedral residual kernels.
#include "fe_device.h"

namespace fe {

LaunchFn select_sumfact(const Plan &) { return nullptr; }

}  // namespace fe

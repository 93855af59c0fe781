// Matrix-core (MFMA) element-matrix kernels.
#include "fe_device.h"

namespace fe {

LaunchFn select_mfma(const Plan &) { return nullptr; }

}  // namespace fe

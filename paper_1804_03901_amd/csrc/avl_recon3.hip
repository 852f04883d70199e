// 1D-3V reconstruction (16-corner cloud-in-cell in x, vx, vy, vz).
#include "avl_device.h"

namespace avl {

size_t recon3_scratch_bytes(const Geo&) { return 0; }

hipError_t launch_recon3(const Geo&, void*, const int*, void*, void*, double*, void*, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace avl

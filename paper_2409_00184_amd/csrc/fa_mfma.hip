// placeholder, replaced by the MFMA decode
#include "fa_device.hpp"
#include "fa_internal.hpp"
namespace fa {
hipError_t launch_decode_mfma(const DecodeLaunch &, int, int, hipStream_t) {
    return hipErrorNotSupported;
}
}  // namespace fa

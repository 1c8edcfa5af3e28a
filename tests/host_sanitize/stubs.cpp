// The two device-side entry points the host precompute calls, for a build
// of the host sources alone (no HIP): the device inspection reports that no
// device is present, and there is no device state to release.
#include <string>

#include "../../paper_2308_16084_amd/csrc/flood_device.hpp"
#include "../../paper_2308_16084_amd/csrc/p2m_internal.hpp"

namespace p2m {

bool device_flood(const FloodInput&, FloodResult&, std::string& err) {
    err = "device inspection: no device in the host-only build";
    return false;
}

void device_release(MeshState&) {}

}  // namespace p2m

// Stand-in for the HIP device in host-only test builds (sanitizer builds of
// the manager, rings and copy pool run on the loopback backend, without the
// HIP runtime): selecting the HIP backend fails at gvm_init.
#include <memory>

#include "device.hpp"

namespace gvm {

std::unique_ptr<Device> make_hip_device() { return nullptr; }

}  // namespace gvm

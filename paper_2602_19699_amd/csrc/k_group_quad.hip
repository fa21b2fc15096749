// Workgroup-per-instance solver for the 37-state synthetic quadruped.
#include "runtime.hpp"

namespace cbic {

const Launcher* launcher_quad(int) { return nullptr; }

}  // namespace cbic

// Planar 3-link arm instantiation of the lane-per-instance solver.
#include "dev_systems.hpp"
#include "lane_launch.hpp"

namespace cbic {

const Launcher* launcher_arm(int precision) {
  return precision ? LaneLaunch<Arm3, float>::get() : LaneLaunch<Arm3, double>::get();
}

}  // namespace cbic

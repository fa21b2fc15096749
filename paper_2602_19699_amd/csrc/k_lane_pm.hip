// Point-mass and linear-quadratic instantiations of the lane-per-instance solver.
#include "dev_systems.hpp"
#include "lane_launch.hpp"

namespace cbic {

const Launcher* launcher_point_mass(int precision) {
  return precision ? LaneLaunch<PointMass, float>::get() : LaneLaunch<PointMass, double>::get();
}

const Launcher* launcher_lq(int n, int m, int precision) {
  if (n == 2 && m == 1) return precision ? LaneLaunch<LinQuad<2, 1>, float>::get() : LaneLaunch<LinQuad<2, 1>, double>::get();
  if (n == 4 && m == 2) return precision ? LaneLaunch<LinQuad<4, 2>, float>::get() : LaneLaunch<LinQuad<4, 2>, double>::get();
  if (n == 6 && m == 3) return precision ? LaneLaunch<LinQuad<6, 3>, float>::get() : LaneLaunch<LinQuad<6, 3>, double>::get();
  return nullptr;
}

}  // namespace cbic

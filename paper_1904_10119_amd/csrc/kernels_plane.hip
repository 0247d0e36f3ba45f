// Fused 2D plane kernels for planes of 16..128 x 16..128 points.
#include "plane_kernel.h"

namespace dft3d {
template <int N1>
static void add_planes_for_rows(std::vector<KernelInfo>& v) {
  v.push_back(kernel_info_plane<N1, 16>());
  v.push_back(kernel_info_plane<N1, 32>());
  v.push_back(kernel_info_plane<N1, 64>());
  v.push_back(kernel_info_plane<N1, 128>());
}
void register_kernels_plane(std::vector<KernelInfo>& v) {
  add_planes_for_rows<16>(v);
  add_planes_for_rows<32>(v);
  add_planes_for_rows<64>(v);
  add_planes_for_rows<128>(v);
}
}  // namespace dft3d

// Real spherical harmonics basis (paper Sec. 3: real SH up to degree 3, the
// (l, m) pair at index l(l+1)+m), shared by the projection and the SH compaction.
#pragma once

#include <hip/hip_runtime.h>

namespace potr {

// Real spherical harmonics with the Condon-Shortley phase in Cartesian form,
// Y_{l,m}(x, y, z) for a unit vector, stored at index l(l+1)+m. The constants are
// K_l^m times the Legendre polynomial coefficients:
//   l=0: 1/(2 sqrt(pi))
//   l=1: sqrt(3/(4 pi))
//   l=2: sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4
//   l=3: sqrt(35/(2 pi))/4, sqrt(105/pi)/2, sqrt(21/(2 pi))/4, sqrt(7/pi)/4, sqrt(105/pi)/4
__device__ inline void sh_basis_d3(double x, double y, double z, int degree, double* Y) {
    Y[0] = 0.28209479177387814;
    if (degree < 1) return;
    const double c1 = 0.4886025119029199;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (degree < 2) return;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792 * x * y;
    Y[5] = -1.0925484305920792 * y * z;
    Y[6] = 0.31539156525252005 * (2.0 * zz - xx - yy);
    Y[7] = -1.0925484305920792 * x * z;
    Y[8] = 0.5462742152960396 * (xx - yy);
    if (degree < 3) return;
    Y[9] = -0.5900435899266435 * y * (3.0 * xx - yy);
    Y[10] = 2.890611442640554 * x * y * z;
    Y[11] = -0.4570457994644658 * y * (4.0 * zz - xx - yy);
    Y[12] = 0.3731763325901154 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -0.4570457994644658 * x * (4.0 * zz - xx - yy);
    Y[14] = 1.445305721320277 * z * (xx - yy);
    Y[15] = -0.5900435899266435 * x * (xx - 3.0 * yy);
}

}  // namespace potr

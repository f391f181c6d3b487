// dynamic.hip -- the dynamic model's movement step (Sec. III-C): every node
// rotates by its angular step and takes the radial step of Algorithm 2,
// reflected at the centre and at the rim.
//
// The radial step is taken on s = sinh^2(alpha r / 2) = (cosh(alpha r) - 1) / 2,
// the coordinate in which Eq. 1's radius density is uniform (on
// [0, sinh^2(alpha R / 2)]), so that a shift folded back by mirror reflection
// keeps the density (Theorem 1).  The step tau_r is given in units of
// cosh(alpha r), i.e. s moves by tau_r / 2; the sinh^2 form keeps full relative
// precision near the centre, where cosh(alpha r) - 1 would cancel.
// One thread per node; the arrays are read and written once.  The step is
// bound by its FP64 sinh and asinh, not by the 48 bytes it moves per node.
#include "rhg_kernels.h"

namespace rhgk {
using namespace rhgd;

__global__ __launch_bounds__(256) void k_move(uint64_t n, double alpha, double R, double S, double *theta, double *r,
                                              const double *tau_phi, double *tau_r) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // rotation, into [0, fl(2 pi)); inside it the quotient's floor is 0 (the
    // rounded quotient of t < fl(2 pi) stays below 1), so the division is skipped
    double t = theta[i] + tau_phi[i];
    if (!(t >= 0.0 && t < TWO_PI)) {
        t = t - TWO_PI * floor(t / TWO_PI);
        if (t >= TWO_PI || t < 0.0) t = 0.0;
    }
    theta[i] = t;
    // radial step: y = s + tau_r / 2 folded into [0, S]; k = floor(y / S)
    // boundary crossings, each a mirror reflection that negates the step
    const double tr = tau_r[i];
    if (tr == 0.0) return;  // a zero step leaves the radius exactly as it is
    const double h = sinh(alpha * r[i] / 2.0);
    const double y = h * h + tr / 2.0;
    double k = 0.0;  // y in [0, S): no crossing (floor of the quotient is 0, as above)
    if (!(y >= 0.0 && y < S)) k = floor(y / S);
    // parity of the integer k: |k| >= 2^53 is even (as fmod(|k|, 2) says)
    const double ak = fabs(k);
    const bool odd = ak < 9007199254740992.0 && (((unsigned long long)ak) & 1ull) != 0ull;
    double s2 = odd ? (k + 1.0) * S - y : y - k * S;
    if (s2 < 0.0) s2 = 0.0;
    if (s2 > S) s2 = S;
    if (odd) tau_r[i] = -tr;
    const double r2 = 2.0 * asinh(sqrt(s2)) / alpha;
    r[i] = r2 > R ? R : r2;
}

void move(uint64_t n, double alpha, double R, double S, double *theta, double *r, const double *tau_phi,
          double *tau_r, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_move, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, alpha, R, S, theta, r,
                       tau_phi, tau_r);
}

}  // namespace rhgk

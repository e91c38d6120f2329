// Orientation predicates used by every walk decision.
//
// orient(a, b, c) = (ax - cx)(by - cy) - (ay - cy)(bx - cx) is twice the
// signed area of (a, b, c); for a counter-clockwise triangle the barycentric
// coordinate of q at vertex k is orient(x_{k+1}, x_{k+2}, q) / (2 area)
// (eq. barycoords), so its sign is the sign of this determinant.
//
// Three stages, each taken only when the previous one cannot certify the
// sign:
//   1. FP32 determinant with the static bound (3u + 16u^2)(|l| + |r|), u = 2^-24
//      (FP32 meshes only);
//   2. FP64 determinant with the same bound for u = 2^-53 (Shewchuk, "Adaptive
//      precision floating-point arithmetic and fast robust geometric
//      predicates", DCG 18, 1997, the static error bound of orient2d);
//   3. the exact sign, from the six coordinate products of the expanded
//      determinant turned into exact two-term products (fused multiply-add)
//      and summed with error-free transformations into a non-overlapping
//      expansion (same paper, Grow-Expansion with zero elimination); the sign
//      of such an expansion is the sign of its largest component.
// The file is compiled with -ffp-contract=off: every expression rounds as
// written, which the bounds of stages 1-2 assume.  Stage 3 first scales all
// six coordinates by 2^150 (exact, and it leaves the sign unchanged: the
// determinant is homogeneous of degree 2).  With mesh coordinates 0 or of
// magnitude in [2^-100, 2^100] and any finite query coordinate inside the
// mesh's bounding box, every nonzero scaled coordinate lies in
// [2^-924, 2^250]; each coordinate product then pairs a mesh value >= 2^50
// with a value >= 2^-924 (or two mesh values), its exponent stays >= -874,
// so its rounding error is a representable double, and no sum overflows:
// stage 3 is exact on that whole domain.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#define SLW_HD __host__ __device__ __forceinline__

namespace slw {

constexpr double kEps64 = 0x1p-53;
constexpr double kBound64 = (3.0 + 16.0 * kEps64) * kEps64;
// covers the absolute rounding of products that land in the subnormal range
constexpr double kAbs64 = 0x1p-1070;
constexpr float kEps32 = 0x1p-24f;
constexpr float kBound32 = (3.0f + 16.0f * kEps32) * kEps32;
constexpr float kAbs32 = 0x1p-146f;
// exactness domain of mesh coordinates (0 or magnitude in [kTinyCoord, kHugeCoord])
constexpr double kTinyCoord = 0x1p-100;
constexpr double kHugeCoord = 0x1p100;
constexpr double kExactScale = 0x1p150;

SLW_HD void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    double bv = s - a;
    double av = s - bv;
    e = (a - av) + (b - bv);
}

SLW_HD void two_prod(double a, double b, double &p, double &e)
{
    p = a * b;
    e = fma(a, b, -p);
}

// Exact sign of ax*by - ax*cy - cx*by - ay*bx + ay*cx + cy*bx
// (the determinant multiplied out; the cx*cy terms cancel).
__host__ __device__ __noinline__ inline int orient_exact_sign(double ax, double ay, double bx, double by,
                                                               double cx, double cy)
{
    ax *= kExactScale;
    ay *= kExactScale;
    bx *= kExactScale;
    by *= kExactScale;
    cx *= kExactScale;
    cy *= kExactScale;
    const double u[6] = {ax, -ax, -cx, -ay, ay, cy};
    const double v[6] = {by, cy, by, bx, cx, bx};
    double h[13];
    int n = 0;
    for (int t = 0; t < 6; ++t) {
        double p, e;
        two_prod(u[t], v[t], p, e);
        const double add[2] = {e, p};
        for (int s = 0; s < 2; ++s) {
            // grow the expansion h[0..n) by add[s], dropping zero components
            double q = add[s];
            int m = 0;
            for (int i = 0; i < n; ++i) {
                double qn, hh;
                two_sum(q, h[i], qn, hh);
                if (hh != 0.0)
                    h[m++] = hh;
                q = qn;
            }
            if (q != 0.0)
                h[m++] = q;
            n = m;
        }
    }
    if (n == 0)
        return 0;
    return h[n - 1] > 0.0 ? 1 : -1;
}

// Stage 2 filter on the two rounded products l = (ax-cx)(by-cy) and
// r = (ay-cy)(bx-cx): returns det = l - r and whether its sign is certain.
SLW_HD double filter64(double l, double r, bool &certain)
{
    double det = l - r;
    double bound = kBound64 * (fabs(l) + fabs(r)) + kAbs64;
    certain = (det > bound) || (-det > bound);
    return det;
}

// Stage 1 filter, same form in float.
SLW_HD float filter32(float l, float r, bool &certain)
{
    float det = l - r;
    float bound = kBound32 * (fabsf(l) + fabsf(r)) + kAbs32;
    certain = (det > bound) || (-det > bound);
    return det;
}

// Stage 2 on its own: the FP64 determinant, and whether its sign is exact.
SLW_HD double orient_fp64(double ax, double ay, double bx, double by, double cx, double cy, bool &certain)
{
    return filter64((ax - cx) * (by - cy), (ay - cy) * (bx - cx), certain);
}

SLW_HD int sign_of(double d) { return (d > 0.0) - (d < 0.0); }

// Exact sign, stages 2-3.
SLW_HD int orient_sign64(double ax, double ay, double bx, double by, double cx, double cy)
{
    bool certain;
    double d = orient_fp64(ax, ay, bx, by, cx, cy, certain);
    if (certain)
        return sign_of(d);
    return orient_exact_sign(ax, ay, bx, by, cx, cy);
}

// The walk's float filter: differences (a~ - q~), (b~ - q~) of inputs that
// were rounded to float (after subtracting a common centre), and the
// coefficients of the error bound derived for that rounding (see
// filter_constants).  Returns +1 / -1 when the sign of the exact determinant
// is certified, 0 when it is not; det receives the float determinant.
//   det = fma(dxa, dyb, -(dya dxb)): one rounding fewer than l - r, so the
//   bound derived for l - r still holds;
//   |l| + |r| <= Sa Sb with Sv = |dxv| + |dyv|, so c1 Sa Sb + c2 (Sa + Sb) + c3
//   is at least the derived bound (the slack in c1, c2 absorbs the
//   rounding of this expression itself).
SLW_HD int filter_sign_f32(float dxa, float dya, float dxb, float dyb, float c1, float c2, float c3, float &det)
{
    det = fmaf(dxa, dyb, -(dya * dxb));
    const float sa = fabsf(dxa) + fabsf(dya);
    const float sb = fabsf(dxb) + fabsf(dyb);
    const float bnd = fmaf(c1, sa * sb, fmaf(c2, sa + sb, c3));
    if (!(fabsf(det) > bnd))
        return 0;
    return det > 0.0f ? 1 : -1;
}

// Exact sign for float inputs, stages 1-3.
SLW_HD int orient_sign32(float ax, float ay, float bx, float by, float cx, float cy)
{
    bool certain;
    float d = filter32((ax - cx) * (by - cy), (ay - cy) * (bx - cx), certain);
    if (certain)
        return (d > 0.0f) - (d < 0.0f);
    return orient_sign64(ax, ay, bx, by, cx, cy);
}

}  // namespace slw

// Elementary functions of the FP32 kernel paths, written for the bounded
// arguments they see (phases of order 1 to 1e3 radians).
#pragma once

#include <hip/hip_runtime.h>

namespace cia {

// sin and cos of an FP32 angle.  Cody-Waite reduction t = q (pi/2) + r with
// pi/2 split into three floats (exact products through FMA; the residual
// is below 1e-21 relative, so |q| up to 2^20 keeps r accurate), then the
// Taylor series of sin (to r^11) and cos (to r^12) on |r| <= pi/4, whose
// truncation errors are below 1e-11, in Horner form; the quadrant q mod 4
// swaps and signs the pair.  Accurate to a few units in the last place.
__host__ __device__ inline void fast_sincosf(float t, float *s, float *c) {
    const float q = rintf(t * 6.36619746685028076172e-01f);
    float r = fmaf(-q, 1.57079637050628662109e+00f, t);
    r = fmaf(-q, -4.37113882867379288655e-08f, r);
    r = fmaf(-q, -1.71512451000588187280e-15f, r);
    const float r2 = r * r;
    float ps = fmaf(r2, -2.50521083854417188e-08f, 2.75573192239858907e-06f);
    ps = fmaf(r2, ps, -1.98412698412698413e-04f);
    ps = fmaf(r2, ps, 8.33333333333333333e-03f);
    ps = fmaf(r2, ps, -1.66666666666666667e-01f);
    const float sr = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, 2.08767569878680990e-09f, -2.75573192239858907e-07f);
    pc = fmaf(r2, pc, 2.48015873015873016e-05f);
    pc = fmaf(r2, pc, -1.38888888888888889e-03f);
    pc = fmaf(r2, pc, 4.16666666666666667e-02f);
    pc = fmaf(r2, pc, -0.5f);
    const float cr = fmaf(r2, pc, 1.0f);
    const int qi = (int)q & 3;
    const float a = (qi & 1) ? cr : sr;
    const float b = (qi & 1) ? sr : cr;
    *s = (qi & 2) ? -a : a;
    *c = ((qi + 1) & 2) ? -b : b;
}

}  // namespace cia

// Double-double (dd) arithmetic on the device: a value is the unevaluated sum hi + lo of
// two doubles with |lo| <= ulp(hi) / 2.  Built from the error-free transformations
// TwoSum (Knuth) and TwoProduct (with the fused multiply-add, exact for doubles without
// overflow or underflow); the compensated dot product is Dot2 of Ogita, Rump & Oishi
// (SIAM J. Sci. Comput. 26, 2005), as accurate as a dot product in twice the precision.
//
// Every function body turns floating-point contraction off: a product fused into the next
// addition (hipcc fuses across statements by default) is not the rounded product the error
// terms are computed for, and the transformations would no longer be error-free.
//
// Used by the step residual ||A f - g|| / ||g||: expanded through scalar products of CP
// tensors its three parts cancel, so in plain FP64 a relative residual below ~1e-8 is
// rounding noise; with every Gram entry, Hadamard product and sum in dd it is resolved
// down to ~1e-15.
#pragma once
#include <hip/hip_runtime.h>

namespace cpals {

struct dd {
    double hi, lo;
};

// a + b = s + e exactly
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// a + b = s + e exactly, |a| >= |b| (or a == 0)
__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
    s = a + b;
    e = b - (s - a);
}

// a b = p + e exactly
__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
#pragma clang fp contract(off)
    p = a * b;
    e = fma(a, b, -p);
}

__device__ __forceinline__ dd dd_from(double a) { return dd{a, 0.0}; }

__device__ __forceinline__ dd dd_add(dd x, dd y) {
#pragma clang fp contract(off)
    double s, e;
    two_sum(x.hi, y.hi, s, e);
    e += x.lo + y.lo;
    dd r;
    fast_two_sum(s, e, r.hi, r.lo);
    return r;
}

__device__ __forceinline__ dd dd_mul(dd x, dd y) {
#pragma clang fp contract(off)
    double p, e;
    two_prod(x.hi, y.hi, p, e);
    e = fma(x.hi, y.lo, fma(x.lo, y.hi, e));
    dd r;
    fast_two_sum(p, e, r.hi, r.lo);
    return r;
}

__device__ __forceinline__ dd dd_mul_d(dd x, double b) {
#pragma clang fp contract(off)
    double p, e;
    two_prod(x.hi, b, p, e);
    e = fma(x.lo, b, e);
    dd r;
    fast_two_sum(p, e, r.hi, r.lo);
    return r;
}

// One step of Dot2: (s, c) accumulates a b (s the running sum, c the running error).
__device__ __forceinline__ void dot2_step(double a, double b, double& s, double& c) {
#pragma clang fp contract(off)
    double p, pe, t, te;
    two_prod(a, b, p, pe);
    two_sum(s, p, t, te);
    s = t;
    c += pe + te;
}

// Normalised dd from the two Dot2 accumulators.
__device__ __forceinline__ dd dot2_result(double s, double c) {
#pragma clang fp contract(off)
    dd r;
    fast_two_sum(s, c, r.hi, r.lo);
    return r;
}

__device__ __forceinline__ dd dd_shfl_down(dd v, int off) {
#pragma clang fp contract(off)
    return dd{__shfl_down(v.hi, off, 64), __shfl_down(v.lo, off, 64)};
}

// Sum over the wave (fixed tree), valid in lane 0.
__device__ __forceinline__ dd dd_wave_sum(dd v) {
#pragma clang fp contract(off)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = dd_add(v, dd_shfl_down(v, off));
    return v;
}

}  // namespace cpals

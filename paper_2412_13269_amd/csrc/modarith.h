// Modular arithmetic on FP64 for primes below 2^50.
//
// Residues are exact integers held in doubles.  CDNA4 runs FP64 FMA at the
// full vector rate, while a 64x64->128-bit integer product needs several
// quarter-rate 32-bit multiplies, so the products below take the
// error-free-transformation route:
//
//   a*b = h + l exactly, with h = fl(a*b) and l = fma(a, b, -h);
//   c   = round-to-nearest of an estimate of a*b/q, off by at most 0.875;
//   r   = fma(-c, q, h) + l = a*b - c*q exactly (|r| < q, an integer < 2^53);
//   r   += q if negative.
//
// Bounds, for a < 2^50 and b < q < 2^50: |h - a*b| <= 2^46, so h - c*q and
// r are integers below 2^51 in magnitude and every step above is exact.  The
// estimate c uses either fl(fl(a*b) * fl(1/q)) (three roundings, error at most
// 2^50 * 3 * 2^-53 = 0.375) or, for a constant b with bq = fl(b/q) prepared in
// advance, fl(a * bq) (two roundings, error at most 0.25).  Either way
// |a*b/q - c| < 1, so one conditional add of q lands r in [0, q).
//
// The first operand may be any integer below 2^50 (it need not be reduced
// modulo q); the second must be below q.  Compiled with -ffp-contract=off so
// that no multiply-add is fused other than the explicit fma calls.
#pragma once
#include <hip/hip_runtime.h>

namespace pfx {

__device__ __forceinline__ double madd(double a, double b, double q) {
    double s = a + b;
    return s >= q ? s - q : s;
}

__device__ __forceinline__ double msub(double a, double b, double q) {
    double s = a - b;
    return s < 0.0 ? s + q : s;
}

__device__ __forceinline__ double mneg(double a, double q) { return a == 0.0 ? 0.0 : q - a; }

// a * b mod q, both operands variable; qinv = fl(1/q).
__device__ __forceinline__ double mmul(double a, double b, double q, double qinv) {
    double h = a * b;
    double l = __builtin_fma(a, b, -h);
    double c = __builtin_rint(h * qinv);
    double r = __builtin_fma(-c, q, h) + l;
    return r < 0.0 ? r + q : r;
}

// a * w mod q for a constant w < q with wq = fl(w / q).
__device__ __forceinline__ double mmulc(double a, double w, double wq, double q) {
    double h = a * w;
    double l = __builtin_fma(a, w, -h);
    double c = __builtin_rint(a * wq);
    double r = __builtin_fma(-c, q, h) + l;
    return r < 0.0 ? r + q : r;
}

// x mod q for an integer 0 <= x < 2^50 (x may exceed q by any factor), and for
// 0 <= x < 8q < 2^53: fl(x * qinv) is then within 2^-50 of x/q < 8, so the floor
// is off by at most one, fma(-c, q, x) is an exact small integer, and the two
// corrections land it in [0, q).
__device__ __forceinline__ double mred(double x, double q, double qinv) {
    double c = __builtin_floor(x * qinv);
    double r = __builtin_fma(-c, q, x);
    r = r < 0.0 ? r + q : r;
    return r >= q ? r - q : r;
}

// ---- signed lazy forms (used inside transforms) ---------------------------
// a*w mod q up to a multiple of q: r = a*w - c*q with |r| <= q, for |a| <= 2^51,
// 0 <= w < q < 2^50, wq = fl(w/q).  Same steps as mmulc without the final
// correction: |h - a*w| <= 2^47 and |c - a*w/q| <= 1, so h - c*q and r are
// integers below 2^52 and exact.  For |a| <= q the bound is |r| <= 0.75 q.
__device__ __forceinline__ double mmulc_lazy(double a, double w, double wq, double q) {
    double h = a * w;
    double l = __builtin_fma(a, w, -h);
    double c = __builtin_rint(a * wq);
    return __builtin_fma(-c, q, h) + l;
}

// a*b mod q up to a multiple of q: r = a*b - c*q with |r| <= 0.875 q, for
// integers |a| < 2^50 and |b| < q < 2^50 of either sign (mmul without its final
// correction: the estimate c is off from a*b/q by at most 0.875, as there).
__device__ __forceinline__ double mmul_lazy(double a, double b, double q, double qinv) {
    double h = a * b;
    double l = __builtin_fma(a, b, -h);
    double c = __builtin_rint(h * qinv);
    return __builtin_fma(-c, q, h) + l;
}

// x mod q into [-q/2, q/2] (up to a rounding tie) for an integer |x| < 2^53.
__device__ __forceinline__ double mred_signed(double x, double q, double qinv) {
    return __builtin_fma(-__builtin_rint(x * qinv), q, x);
}

// [0, q) from an integer |x| <= q.
__device__ __forceinline__ double mcanon(double x, double q) {
    x = x < 0.0 ? x + q : x;
    return x >= q ? x - q : x;
}

}  // namespace pfx

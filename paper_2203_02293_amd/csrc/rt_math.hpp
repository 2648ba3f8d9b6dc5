// rt_math.hpp -- small math kernels of the solve, host- and device-callable.
//
// exp_em1(x), FP64: e^x and e^x - 1 from one argument reduction (Cody-Waite
// reduction x = k ln2 + r with |r| <= ln2/2, Taylor polynomial of e^r - 1,
// scaling by 2^k; Tang, ACM TOMS 15 (1989) describes the same structure).
// The expm1 value keeps full relative accuracy near x = 0 because the
// polynomial carries e^r - 1 without its leading 1, and e^x - 1 is rebuilt
// as 2^k (e^r - 1) + (2^k - 1), where 2^k - 1 is exact.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace rtk {

template <class R> struct ExpCfg;
template <> struct ExpCfg<double> {
    static constexpr int DEG = 12;   // |r|^13/13! < 2e-16 for |r| <= ln2/2
    static constexpr double LN2_HI = 6.93147180369123816490e-01;  // 32 leading bits of ln 2
    static constexpr double LN2_LO = 1.90821492927058770002e-10;  // ln 2 - LN2_HI
    static constexpr double LOG2E = 1.44269504088896338700e+00;
    static constexpr double XMAX = 709.0, XMIN = -745.0;
};
template <> struct ExpCfg<float> {
    static constexpr int DEG = 7;    // |r|^8/8! < 2e-8
    static constexpr float LN2_HI = 0.693145751953125f;          // 16 leading bits of ln 2
    static constexpr float LN2_LO = 1.428606765330187045e-06f;
    static constexpr float LOG2E = 1.44269504088896338700f;
    static constexpr float XMAX = 88.0f, XMIN = -104.0f;
};

constexpr double inv_fact(int n)
{
    double f = 1.0;
    for (int m = 2; m <= n; ++m) f *= m;
    return 1.0 / f;
}


// sum_{j=0}^{N-1} C::coef(j) y^j as two interleaved Horner chains in y^2
// (even and odd powers), halving the dependent chain; coefficients folded at
// compile time.
template <class R, class C, int J, int N>
__host__ __device__ __forceinline__ R horner_y2(R y2)
{
    constexpr double cj = C::coef(J);
    if constexpr (J + 2 >= N) {
        return R(cj);
    } else {
        return fma(horner_y2<R, C, J + 2, N>(y2), y2, R(cj));
    }
}

template <class R, class C, int N>
__host__ __device__ __forceinline__ R poly_eo(R y)
{
    if constexpr (N == 1) {
        return R(C::coef(0));
    } else {
        const R y2 = y * y;
        return fma(horner_y2<R, C, 1, N>(y2), y, horner_y2<R, C, 0, N>(y2));
    }
}

// FP64 sum_{j=J}^{N-1} C::coef(j) y^(j-J) as one Horner chain of three-operand
// v_fma_f64 whose coefficients are scalar operands, so no coefficient takes a
// vector register or a vector move (written as fma() with a literal, each step
// compiles to a 64-bit copy of the coefficient into the accumulator and the
// two-operand v_fmac_f64).  z is an opaque zero (opaque_zero()): each
// coefficient is built as its two 32-bit halves XOR z, one scalar instruction
// with a literal operand per half, at its use.  As plain constants, the
// coefficients of the loop body's chains (about 80 distinct doubles in the
// Planck edges alone, more than the scalar registers hold) are hoisted out of
// the loops and spilled, and come back through vector-lane moves, which issue
// as vector instructions.  Same operation, same rounding.
template <class C, int J, int N>
__host__ __device__ __forceinline__ double horner_s(double y, uint32_t z)
{
    constexpr double cj = C::coef(J);
    if constexpr (J + 1 >= N) {
        return cj;
    } else {
        const double p = horner_s<C, J + 1, N>(y, z);
#if defined(__HIP_DEVICE_COMPILE__)
        constexpr uint64_t b = __builtin_bit_cast(uint64_t, cj);
        const double c = __builtin_bit_cast(double, ((uint64_t)(z ^ (uint32_t)(b >> 32)) << 32) |
                                                        (uint64_t)(z ^ (uint32_t)b));
        double out;
        asm("v_fma_f64 %0, %1, %2, %3" : "=v"(out) : "v"(p), "v"(y), "s"(c));
        return out;
#else
        (void)z;
        return fma(p, y, cj);
#endif
    }
}

// A zero the compiler cannot see through, new at every call (so that nothing
// computed from it is hoisted out of a loop or shared between calls).
__host__ __device__ __forceinline__ uint32_t opaque_zero()
{
    uint32_t z = 0;
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(z));
#endif
    return z;
}

// The polynomial by two chains in FP32 (shorter dependent chains); in FP64 by
// one (each extra FP64 partial sum takes two registers, which the FP64 kernel
// does not have to spare), with scalar coefficients.
template <class R, class C, int N>
__host__ __device__ __forceinline__ R poly(R y)
{
    if constexpr (sizeof(R) == 4) return poly_eo<R, C, N>(y);
    else return horner_s<C, 0, N>(y, opaque_zero());
}

// coefficients 1/(j+1)! of (e^r - 1)/r
struct ExpTailCoef {
    static constexpr double coef(int j) { return inv_fact(j + 1); }
};

template <class R>
struct ExpEm1 {
    R e;     // e^x
    R em1;   // e^x - 1
};

template <class R>
__host__ __device__ __forceinline__ ExpEm1<R> exp_em1(R x)
{
    using Cfg = ExpCfg<R>;
    ExpEm1<R> out;
    if (!(x > Cfg::XMIN)) {          // underflow (and -inf): e^x = 0
        out.e = R(0);
        out.em1 = R(-1);
        return out;
    }
    if (x > Cfg::XMAX) x = Cfg::XMAX;
    R k = rint(x * Cfg::LOG2E);
    R r = fma(-k, R(Cfg::LN2_HI), x);
    r = fma(-k, R(Cfg::LN2_LO), r);
    // q = e^r - 1 = r (1 + r/2 + r^2/6 + ...)
    R q = r * poly<R, ExpTailCoef, Cfg::DEG>(r);
    int ki = int(k);
    out.e = ldexp(R(1) + q, ki);
    out.em1 = ldexp(q, ki) + (ldexp(R(1), ki) - R(1));
    return out;
}

// FP32: 2^(x log2 e) from the hardware base-2 exponential (within one ulp),
// with the rounding error of the product x log2 e (an FMA residual plus the
// low part of log2 e) applied as the first-order factor 1 + err ln 2.
// e^x - 1: for |x| < 1/2 the Taylor polynomial x (1 + x/2 + ... + x^7/8!)
// (next term below 6e-9 of x), else e^x - 1 itself, which is then at least
// 0.39 in magnitude (a few ulp).  Arguments below -104 give 0 and -1; no
// branches, so the lanes of a wavefront never diverge here.
struct ExpTail8 {
    static constexpr double coef(int j) { return inv_fact(j + 1); }
};

template <>
__host__ __device__ __forceinline__ ExpEm1<float> exp_em1<float>(float x)
{
    constexpr float L = 1.44269502162933349609375f;                // log2 e rounded to FP32
    constexpr float LLO = float(1.44269504088896340736 - 1.44269502162933349609375);
    constexpr float LN2 = 0.693147180559945309f;
    x = fminf(fmaxf(x, -104.0f), 88.0f);
    const float y = x * L;
    const float yl = fmaf(x, LLO, fmaf(x, L, -y));
#if defined(__HIP_DEVICE_COMPILE__)
    const float e0 = __builtin_amdgcn_exp2f(y);
#else
    const float e0 = exp2f(y);
#endif
    ExpEm1<float> out;
    out.e = fmaf(e0, yl * LN2, e0);
    const float q = x * poly_eo<float, ExpTail8, 8>(x);
    out.em1 = fabsf(x) < 0.5f ? q : out.e - 1.0f;
    return out;
}

// e^x in FP32 for an FP64 argument: the FP32 exponential of the rounded
// argument, times 1 + (its rounding error).  A large argument thus keeps the
// relative accuracy of FP32 (an argument rounded to FP32 costs |x| 2^-24 of
// e^x: 4e-6 at x = -70, a Wien-tail Planck edge of a cold column).
__host__ __device__ __forceinline__ ExpEm1<float> exp_em1_f(double x)
{
    x = fmin(fmax(x, -104.0), 88.0);
    const float xh = float(x);
    const float xl = float(x - double(xh));
    ExpEm1<float> e = exp_em1(xh);
    e.em1 = fmaf(e.e, xl, e.em1);
    e.e = fmaf(e.e, xl, e.e);
    return e;
}

// 1/x: the hardware reciprocal (relative error below 5e-8 on gfx950) refined
// by one Newton step, which squares the error: within about 2e-15 (measured
// 2.1e-15 over 2^20 arguments spanning e^-12..e^12), ten ulp at most.
__host__ __device__ __forceinline__ double rcp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
#else
    return 1.0 / x;
#endif
}

// FP32: the hardware reciprocal alone (within one ulp), enough for the FP32
// coefficient build.
__host__ __device__ __forceinline__ float rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// 1/sqrt(x) of a positive finite argument: in FP32 the hardware instruction
// (within one ulp); in FP64 the hardware estimate refined by two Newton steps
// y (3 - x y^2) / 2, each squaring the relative error.
__host__ __device__ __forceinline__ float rsqrt_pos(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}

__host__ __device__ __forceinline__ double rsqrt_pos(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    return y * fma(-hx * y, y, 1.5);
#else
    return 1.0 / sqrt(x);
#endif
}

// A value that is the same in every lane of the wavefront, moved to a scalar
// register so that branches on it are uniform.
__host__ __device__ __forceinline__ int wave_uniform(int x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_readfirstlane(x);
#else
    return x;
#endif
}

}  // namespace rtk

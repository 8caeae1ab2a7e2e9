// Device evaluation of the scan temperature: superposed moving point sources
// on the adiabatic surface of a semi-infinite body (linear conduction), each
// switched on at t_on and off after dur, clamped at T_clamp.  This replaces
// the paper's FEM heat solve (Sec. 2.1) as the driver of the phase update.
//
// For a source of absorbed power q, speed v, on for tau, the rise at a point a
// distance R from the current source position and xi ahead of it along the
// motion is
//   F = q/(4 pi k R) [ e^{-v(xi+R)/(2 alpha)} erfc((R - v tau)/s)
//                    + e^{-|x - P0|^2/(4 alpha tau)} erfcx((R + v tau)/s) ],
// s = 2 sqrt(alpha tau), P0 the start point (time integral of instantaneous
// point sources; the second term is written with erfcx so that nothing
// overflows).  A switched-off track subtracts the same expression for a
// virtual source started at its end point dur later (same current position).
//
// Coordinates are in grid units relative to the grid origin.  The host splits
// each source position into an integer and a fractional part so that the
// offset point - source keeps full float32 relative precision at any
// distance.  erfc/erfcx use the Chebyshev-fitted form of Numerical Recipes
// (Press et al., 2nd ed., Sec. 6.2, "erfcc": relative error below 1.2e-7):
//   erfc(z) = t exp(-z^2 + P(t)), t = 1/(1 + z/2), z >= 0.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phase_model.h"

namespace mstruct {

// one window slot of the scan at one time point (64 bytes)
struct SrcRec {
    int32_t ix, iy, iz;  // integer part of the current source position [grid units]
    float fx, fy, fz;    // fractional part
    float ux, uy;        // unit direction of motion
    float lamp;          // log2(q / (4 pi k h)) [K grid]; -inf marks an unused slot
    float c1;            // v h / (2 alpha) log2(e)
    float vt;            // v tau / h
    float is;            // h / (2 sqrt(alpha tau))
    float e2;            // h^2 / (4 alpha tau) log2(e)
    float vt1, is1, e21; // same for tau - dur of a switched-off track; is1 = 0 while on
};
static_assert(sizeof(SrcRec) == 64, "SrcRec layout");

// P(t) of the erfcc form, converted to base 2: returns log2(e) P(t)
__device__ __forceinline__ float erfc_poly_log2(float t) {
    float p = fmaf(t, 0.17087277f, -0.82215223f);
    p = fmaf(t, p, 1.48851587f);
    p = fmaf(t, p, -1.13520398f);
    p = fmaf(t, p, 0.27886807f);
    p = fmaf(t, p, -0.18628806f);
    p = fmaf(t, p, 0.09678418f);
    p = fmaf(t, p, 0.37409196f);
    p = fmaf(t, p, 1.00002368f);
    p = fmaf(t, p, -1.26551223f);
    return p * kLog2e;
}

// exp2(lg) * erfc(|y|) for any y, i.e. the small part of erfc; the caller adds
// 2 e^{...} for negative y.  lg is an extra base-2 exponent folded in.
__device__ __forceinline__ float scaled_erfc_abs(float y, float lg) {
    const float z = fabsf(y);
    const float t = frcp(fmaf(0.5f, z, 1.0f));
    return t * fexp2(fmaf(-z * z, kLog2e, erfc_poly_log2(t)) + lg);
}

// exp2(lg) * erfcx(y) for y >= 0
__device__ __forceinline__ float scaled_erfcx(float y, float lg) {
    const float t = frcp(fmaf(0.5f, y, 1.0f));
    return t * fexp2(erfc_poly_log2(t) + lg);
}

// A term whose magnitude is provably below 1e-4 K is dropped: every term is
// rR * (factor <= 2) * 2^(lg + lamp) with rR = 1/R <= 2^(-(e-1)/2) when
// R^2 = f 2^e, f in [0.5, 1).  The small part E(|y|) of an erfc is bounded by
// e^{-y^2} (erfc(z) <= e^{-z^2} for z >= 0) and dropped on the same test.  Up
// to four dropped terms per slot (E1, Eb, the two start-point terms, or the
// whole leading term) change T by less than 4e-4 K.
constexpr float kLog2DropK = -13.2877f;  // log2(1e-4)

// Contribution of one slot at grid point (gi, gj, gk) (z grid coordinate -gk).
// Returns +inf when the point is within sqrt(r2min) of a switched-on source
// (the clamp applies).  A switched-off track is the difference of two sources
// sharing a virtual current position; its field is smooth there, but the
// closed form is 0/0 at it, so within roff of that position the contribution
// is taken roff below it.
__device__ __forceinline__ float source_rise(const SrcRec& s, int gi, int gj, int gk, float r2min, float roff) {
    float dx = (float)(gi - s.ix) - s.fx;
    float dy = (float)(gj - s.iy) - s.fy;
    float dz = (float)(-gk - s.iz) - s.fz;
    float R2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    if (s.is1 > 0.0f) {
        if (R2 < roff * roff) {
            dx = 0.0f;
            dy = 0.0f;
            dz = -roff;
            R2 = roff * roff;
        }
    } else if (R2 < r2min) {
        return __builtin_inff();
    }
    const float rR = __builtin_amdgcn_rsqf(R2);
    const float R = R2 * rR;
    const float xi = fmaf(dx, s.ux, dy * s.uy);
    const float cr = fmaf(dx, s.uy, -dy * s.ux);  // in-plane offset across the track
    const float rho2 = fmaf(cr, cr, dz * dz);
    // threshold on lg + lamp below which a term is negligible
    const float cut = kLog2DropK - 1.0f + 0.5f * (float)(__builtin_amdgcn_frexp_expf(R2) - 1);
    // xi + R without cancellation behind the source: rho^2 / (R - xi)
    const float xr = xi >= 0.0f ? xi + R : rho2 * frcp(R - xi);
    const float lg1 = fmaf(-s.c1, xr, s.lamp);  // log2 of amp e^{-v(xi+R)/(2 alpha)}

    // leading term e1 erfc(y1) of the source switched on at P0, minus
    // e1 erfc(y1b) of the virtual source after switch-off; erfc(y) is split
    // as base + sign * E(|y|) with base 2 for y < 0, so that equal bases
    // cancel exactly
    float acc = 0.0f;
    if (lg1 > cut) {
        const float y1 = (R - s.vt) * s.is;
        const bool n1 = y1 < 0.0f;
        float base = n1 ? 2.0f : 0.0f;
        if (fmaf(-y1 * y1, kLog2e, lg1) > cut) {
            const float E1 = scaled_erfc_abs(y1, lg1);
            acc = n1 ? -E1 : E1;
        }
        if (s.is1 > 0.0f) {
            const float y1b = (R - s.vt1) * s.is1;
            const bool nb = y1b < 0.0f;
            if (fmaf(-y1b * y1b, kLog2e, lg1) > cut) {
                const float Eb = scaled_erfc_abs(y1b, lg1);
                acc -= nb ? -Eb : Eb;
            }
            base -= nb ? 2.0f : 0.0f;
        }
        if (base != 0.0f) acc = fmaf(base, fexp2(lg1), acc);
    }
    // start-point terms (erfcx <= 1)
    {
        const float d = xi + s.vt;
        const float lg2 = fmaf(-s.e2, fmaf(d, d, rho2), s.lamp);
        if (lg2 > cut) acc += scaled_erfcx((R + s.vt) * s.is, lg2);
    }
    if (s.is1 > 0.0f) {
        const float d = xi + s.vt1;
        const float lg2 = fmaf(-s.e21, fmaf(d, d, rho2), s.lamp);
        if (lg2 > cut) acc -= scaled_erfcx((R + s.vt1) * s.is1, lg2);
    }
    return rR * acc;
}

// One track over the time points of one launch (a K-step block): its
// current (or, after switch-off, virtual) position at the first and at the
// last time point where it is in the window, and the slot constants at the
// last one, where each drop test of source_rise is least strict (64 bytes).
struct EnvRec {
    float px, py, pz;  // position at the last time point [grid units from the origin]
    float qx, qy;      // position at the first time point (same z)
    float ux, uy;      // unit direction of motion
    float lamp, c1;    // as in SrcRec
    float e2, vt;      // at the last time point (e2 is smallest there)
    float e21, vt1;    // at the last time point if the track is then switched off, else 0
    float is;          // as in SrcRec, at the last time point (is is smallest there)
    float pad[2];
};
static_assert(sizeof(EnvRec) == 64, "EnvRec layout");

// Distances from grid point (gi, gj, gk) to one track over the time points an
// EnvRec covers.  Over a launch the current (or virtual) position moves along
// the straight segment from (qx, qy) to (px, py), so R is at least the
// distance to that segment; along the motion xi only decreases, so xi + R is
// smallest at the last position; the start-point distance |x - P0| is fixed.
struct EnvGeom {
    float Rmin2;  // 0.99 x the squared distance to the segment (a lower bound of R^2 at every time point)
    float xi;     // along the motion from the last position
    float rho2;   // squared distance from the line of motion
    float xr;     // xi + R at the last position (a lower bound over the launch)
};

__device__ __forceinline__ EnvGeom env_geometry(const EnvRec& e, int gi, int gj, int gk) {
    const float x = (float)gi, y = (float)gj, dz = (float)(-gk) - e.pz;
    const float dx = x - e.px, dy = y - e.py;
    EnvGeom g;
    g.xi = fmaf(dx, e.ux, dy * e.uy);
    const float cr = fmaf(dx, e.uy, -dy * e.ux);
    g.rho2 = fmaf(cr, cr, dz * dz);
    const float R2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float qx = x - e.qx, qy = y - e.qy;
    const float xi0 = fmaf(qx, e.ux, qy * e.uy);
    const float R02 = fmaf(qx, qx, fmaf(qy, qy, dz * dz));
    g.Rmin2 = 0.99f * ((xi0 >= 0.0f && g.xi <= 0.0f) ? g.rho2 : fminf(R2, R02));
    const float R = R2 * __builtin_amdgcn_rsqf(R2);
    g.xr = g.xi >= 0.0f ? g.xi + R : g.rho2 * frcp(R - g.xi);
    return g;
}

// True if, at grid point (gi, gj, gk), source_rise drops every term of this
// track at every time point the record covers, so that the track adds
// exactly 0 to T there.  Each bound follows a drop test of source_rise, with
// the distances of env_geometry and e2, e21 (which only decrease) at the last
// time point; R is at least sqrt(Rmin2), which bounds the threshold from
// below.  rlim2 >= 1 keeps the point outside the clamp radius and the
// switched-off offset radius of source_rise.  1 % of R^2, 0.25 in the base-2
// exponents and 0.1 % of the exponents' distances cover float32 rounding of
// both computations (and the hardware rsq and rcp here).
__device__ __forceinline__ bool env_negligible(const EnvRec& e, int gi, int gj, int gk, float rlim2) {
    const EnvGeom g = env_geometry(e, gi, gj, gk);
    if (!(g.Rmin2 >= rlim2)) return false;
    const float cut = kLog2DropK - 1.25f + 0.5f * (float)(__builtin_amdgcn_frexp_expf(g.Rmin2) - 1);
    if (fmaf(-e.c1, 0.999f * g.xr, e.lamp) > cut) return false;
    const float s0 = g.xi + e.vt;
    if (fmaf(-e.e2, 0.999f * fmaf(s0, s0, g.rho2), e.lamp) > cut) return false;
    if (e.e21 > 0.0f) {
        const float s1 = g.xi + e.vt1;
        if (fmaf(-e.e21, 0.999f * fmaf(s1, s1, g.rho2), e.lamp) > cut) return false;
    }
    return true;
}

// An upper bound of source_rise of this track at (gi, gj, gk) at every time
// point the record covers (+inf if the point may come within rlim2 of it).
// The leading term is 2^lg1 / R times a difference of erfc values in
// [0, 2], and at most 2^lg1 e^{-y^2} / R when y = (R - v tau) s^-1 >= 0
// (erfc(y) <= e^{-y^2}; a switched-off track only subtracts from it); y is
// bounded below with R >= sqrt(Rmin2), v tau at most vt and 1/s at least is
// of the last time point.  The start-point term is at most 2^lg2 / R
// (erfcx <= 1 for a non-negative argument), and a switched-off track's
// end-point term is subtracted.  The margins cover float32 rounding of both
// computations and the 1.2e-7 relative error of the erfc form.
__device__ __forceinline__ float env_rise_bound(const EnvRec& e, int gi, int gj, int gk, float rlim2) {
    const EnvGeom g = env_geometry(e, gi, gj, gk);
    if (!(g.Rmin2 >= rlim2)) return __builtin_inff();
    const float rR = __builtin_amdgcn_rsqf(g.Rmin2);
    const float lg1 = fmaf(-e.c1, 0.999f * g.xr, e.lamp);
    const float y = fmaf(g.Rmin2, rR, -e.vt) * e.is;
    const float t1 = y > 0.0f ? fexp2(fmaf(-0.999f * y * y, kLog2e, lg1)) : 2.0f * fexp2(lg1);
    const float s0 = g.xi + e.vt;
    const float t2 = fexp2(fmaf(-e.e2, 0.999f * fmaf(s0, s0, g.rho2), e.lamp));
    return 1.002f * rR * (t1 + t2);
}

// An axis-aligned box of grid positions (x = i, y = j, z = -k).
struct GridBox {
    float xl, xh, yl, yh, zl, zh;
};

// distance from [lo, hi] to c along one axis: nearest and farthest
__device__ __forceinline__ float axis_near(float lo, float hi, float c) { return fmaxf(0.0f, fmaxf(lo - c, c - hi)); }
__device__ __forceinline__ float axis_far(float lo, float hi, float c) { return fmaxf(fabsf(lo - c), fabsf(hi - c)); }

// env_rise_bound for every point of a box at once: the same terms, with the
// distances bounded over the box.  R is at least the distance from the box
// to the bounding box of the segment Q..P.  For d = x - P, xi + R is |d| or
// more where d points along the motion, and rho^2 / (|d| - xi) >=
// rho^2 / (2 |d|) behind it, so it is at least the smaller of the least |d|
// and the least rho^2 over twice the largest |d| (rho is the distance from
// the line of motion, whose cross-track part is linear in x and y and is
// bounded at the corners).  |x - P0|, P0 = P - vt u the start point, is at
// least the distance from the box to P0.
__device__ __forceinline__ float env_box_rise_bound(const EnvRec& e, const GridBox& b, float rlim2) {
    // gap between the box and the segment's bounding box along each axis
    const float gx = fmaxf(0.0f, fmaxf(fminf(e.qx, e.px) - b.xh, b.xl - fmaxf(e.qx, e.px)));
    const float gy = fmaxf(0.0f, fmaxf(fminf(e.qy, e.py) - b.yh, b.yl - fmaxf(e.qy, e.py)));
    const float nz = axis_near(b.zl, b.zh, e.pz);
    const float Rmin2 = 0.99f * fmaf(gx, gx, fmaf(gy, gy, nz * nz));
    // (P is inside the segment's bounding box, so below dmin2 >= Rmin2 >= 1)
    if (!(Rmin2 >= rlim2)) return __builtin_inff();
    const float nx = axis_near(b.xl, b.xh, e.px), ny = axis_near(b.yl, b.yh, e.py);
    const float fx = axis_far(b.xl, b.xh, e.px), fy = axis_far(b.yl, b.yh, e.py), fz = axis_far(b.zl, b.zh, e.pz);
    const float dmin2 = 0.99f * fmaf(nx, nx, fmaf(ny, ny, nz * nz));
    const float dmax2 = 1.01f * fmaf(fx, fx, fmaf(fy, fy, fz * fz));
    // cross-track offset dx uy - dy ux at the four corners
    const float xl = b.xl - e.px, xh = b.xh - e.px, yl = b.yl - e.py, yh = b.yh - e.py;
    const float c0 = fmaf(xl, e.uy, -yl * e.ux), c1 = fmaf(xl, e.uy, -yh * e.ux);
    const float c2 = fmaf(xh, e.uy, -yl * e.ux), c3 = fmaf(xh, e.uy, -yh * e.ux);
    const float cmin = fminf(fminf(c0, c1), fminf(c2, c3)), cmax = fmaxf(fmaxf(c0, c1), fmaxf(c2, c3));
    const float cr = (cmin <= 0.0f && cmax >= 0.0f) ? 0.0f : 0.99f * fminf(fabsf(cmin), fabsf(cmax));
    const float rho2 = fmaf(cr, cr, nz * nz);
    const float xr = fminf(dmin2 * __builtin_amdgcn_rsqf(dmin2), 0.5f * rho2 * __builtin_amdgcn_rsqf(dmax2));
    const float rR = __builtin_amdgcn_rsqf(Rmin2);
    const float lg1 = fmaf(-e.c1, 0.999f * fmaxf(xr, 0.0f), e.lamp);
    const float y = fmaf(Rmin2, rR, -e.vt) * e.is;
    const float t1 = y > 0.0f ? fexp2(fmaf(-0.999f * y * y, kLog2e, lg1)) : 2.0f * fexp2(lg1);
    const float ax = axis_near(b.xl, b.xh, fmaf(-e.vt, e.ux, e.px)), ay = axis_near(b.yl, b.yh, fmaf(-e.vt, e.uy, e.py));
    const float d02 = 0.99f * fmaf(ax, ax, fmaf(ay, ay, nz * nz));
    const float t2 = fexp2(fmaf(-e.e2, 0.999f * d02, e.lamp));
    return 1.002f * rR * (t1 + t2);
}

// all points of the calling wave certified cold for the launch: every track
// of env drops out at every one of them (inactive lanes count as cold).
// n_env < 0: no certificate, every wave evaluates the temperature.
__device__ __forceinline__ bool wave_cold(const EnvRec* __restrict__ env, int n_env, bool act, int gi, int gj,
                                          int gk, float rlim2) {
    if (n_env < 0) return false;
    bool cold = true;
    if (act)
        for (int e = 0; e < n_env && cold; ++e) cold = env_negligible(env[e], gi, gj, gk, rlim2);
    return __ballot(!cold) == 0;
}

// all points of the calling wave certified to stay below Tlim at every time
// point of the launch: T0 plus the rise bound of every track of env is below
// it (inactive lanes pass).  The caller checks n_env >= 0.
__device__ __forceinline__ bool wave_below(const EnvRec* __restrict__ env, int n_env, bool act, int gi, int gj,
                                           int gk, float rlim2, float T0, float Tlim) {
    float T = T0;
    if (act)
        for (int e = 0; e < n_env && T < Tlim; ++e) T += env_rise_bound(env[e], gi, gj, gk, rlim2);
    return __ballot(act && !(T < Tlim)) == 0;
}

template <int W>
__device__ __forceinline__ float scan_temperature(const SrcRec* __restrict__ recs, int gi, int gj, int gk,
                                                  float T0, float Tclamp, float r2min, float roff) {
    float T = T0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const SrcRec s = recs[w];
        if (s.lamp > -1e30f) T += source_rise(s, gi, gj, gk, r2min, roff);
    }
    return fminf(T, Tclamp);
}

}  // namespace mstruct

// Device-side building blocks shared by the kernels: periodic pair geometry,
// cell coordinates, the LJ pair force, reciprocal, and deterministic wave /
// workgroup sums.  Method: tinyMD (arXiv 2009.07400), Sec. 3.2 Eq. 2 and the
// compute_potential example of Sec. 4.2.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace tmd {

// Minimum-image difference along one axis: shift d by one box length when
// |d| > L/2 (positions lie within a fraction of a cell of [0, L), so one
// shift suffices).
__device__ __forceinline__ double mic(double d, double L, double halfL) {
    d = (d > halfL) ? d - L : d;
    d = (d < -halfL) ? d + L : d;
    return d;
}

// |d|^2 summed left to right without fused multiply-add, so that the
// comparison against cutoff^2 and (cutoff + skin)^2 takes the same decision
// as any other IEEE evaluation of dx*dx + dy*dy + dz*dz in that order.
__device__ __forceinline__ double dist2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    return dx * dx + dy * dy + dz * dz;
}

// Pair difference vector with periodic images.  Only atoms near a face of
// the box have partners across it; for every other pair the raw difference
// already is the minimum image.  Any axis with |d| > L/2 makes the raw
// |d|^2 exceed (L/2)^2, so that one comparison selects every pair that may
// need a shift; the correction sits behind a branch that a wavefront takes
// only when one of its lanes needs it, and applies mic() per axis (which
// leaves axes with |d| <= L/2 untouched), so the result is bit-identical to
// applying mic() to every pair.
__device__ __forceinline__ double pair_delta(double xi, double yi, double zi, double xj, double yj, double zj,
                                            double L, double halfL, double halfL2, double &dx, double &dy,
                                            double &dz) {
    dx = xi - xj;
    dy = yi - yj;
    dz = zi - zj;
    double s = dist2(dx, dy, dz);
    if (s >= halfL2) {
        dx = mic(dx, L, halfL);
        dy = mic(dy, L, halfL);
        dz = mic(dz, L, halfL);
        s = dist2(dx, dy, dz);
    }
    return s;
}

// Difference along one axis to the partner's nearest image, xi - (xj + n L)
// with n = rint((xi - xj) / L) in {-1, 0, 1} (positions stay within a
// fraction of a cell of [0, L)): n L is exact, so the shifted partner xj +/-
// L is rounded once, as nearest_image() rounds it.  The shift differs from a
// test of |xi - xj| > L/2 only where (xi - xj) / L rounds across 1/2, that is
// |xi - xj| within an ulp or two of L/2, beyond every cutoff (the library
// requires cutoff + skin < L/2), where the pair adds nothing either way.
__device__ __forceinline__ double mic_delta(double xi, double xj, double L, double invL) {
    return xi - fma(rint((xi - xj) * invL), L, xj);
}

// The pair geometry of the kernels that evaluate forces and their
// derivatives, with |d|^2 formed by fused multiply-adds: there it only
// decides the cutoff test, and the force kernel and the adjoint's
// Hessian-vector product must take that decision identically.  The
// difference is taken to the partner's nearest image (mic_delta()), the
// same two roundings as in pair_delta_img() on a neighborhood copy whose
// positions were moved to their images near the block (see
// nearest_image()), so both give the same bits.  Branch-free: in small
// boxes most wavefronts have a lane whose partner lies across a face.
__device__ __forceinline__ double pair_delta_fma(double xi, double yi, double zi, double xj, double yj, double zj,
                                                double L, double invL, double &dx, double &dy, double &dz) {
    dx = mic_delta(xi, xj, L, invL);
    dy = mic_delta(yi, yj, L, invL);
    dz = mic_delta(zi, zj, L, invL);
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

// pair_delta_fma() for a partner position that already is the image nearest
// to xi: the plain difference.
__device__ __forceinline__ double pair_delta_img(double xi, double yi, double zi, double xj, double yj, double zj,
                                                double &dx, double &dy, double &dz) {
    dx = xi - xj;
    dy = yi - yj;
    dz = zi - zj;
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

// Image of coordinate x (in [0, L)) nearest to c: x shifted by one box
// length when |x - c| > L/2.  A neighborhood copied this way around its
// block's center holds, for every atom i of the block and every list partner
// j, the image of j nearest to i - provided the box has at least E + 4 cells
// per axis and atoms move less than a third of cutoff + skin between list
// builds: then |image - c| <= E a / 2 + (cutoff + skin) + 3 drift < L / 2
// for cells of side a >= cutoff + skin.  With E + 3 cells the bound holds
// for drifts below (3 a / 2 - cutoff - skin) / 3; the pair loops then check
// each difference (engine.hip, pair_geom).
__device__ __forceinline__ double nearest_image(double x, double c, double L, double halfL) {
    const double d = x - c;
    return x + ((d > halfL) ? -L : ((d < -halfL) ? L : 0.0));
}

// 1/s for s > 0: hardware reciprocal estimate refined by one Newton-Raphson
// step r <- r + r (1 - s r), which squares the estimate's relative error
// (about 2^-23 or better) to about 2^-46, far inside the 1e-12 per-atom
// force tolerance.  recip_exact() adds a second step (within an ulp or two
// of the correctly rounded value) for the derivative kernels.
__device__ __forceinline__ double recip(double s) {
    const double r = __builtin_amdgcn_rcp(s);
    return fma(r, fma(-s, r, 1.0), r);
}

__device__ __forceinline__ double recip_exact(double s) {
    const double r = recip(s);
    return fma(r, fma(-s, r, 1.0), r);
}

// Wrap a coordinate less than one box length outside [0, L) into [0, L)
// (a tiny negative p, for which p + L rounds to L, maps to 0), so that
// wrapping twice changes nothing.
__device__ __forceinline__ double wrap(double p, double L) {
    if (p >= L)
        p -= L;
    if (p < 0.0) {
        p += L;
        if (p >= L)
            p = 0.0;
    }
    return p;
}

// Cell index along one axis, clamped to [0, nc) (also for NaN input).
__device__ __forceinline__ int cell_coord(double p, double side, int nc) {
    double q = floor(p / side);
    if (!(q >= 0.0))
        q = 0.0;
    if (q > double(nc - 1))
        q = double(nc - 1);
    return int(q);
}

// Subcell index along one axis (cells cut in halves of side hs = side / 2),
// clamped to [0, 2 nc).  hs is side scaled by a power of two, so p / hs is
// exactly 2 (p / side) and the subcell's cell, the index >> 1, is
// cell_coord(p, side, nc).
__device__ __forceinline__ int sub_coord(double p, double hs, int nc) {
    double q = floor(p / hs);
    if (!(q >= 0.0))
        q = 0.0;
    if (q > double(2 * nc - 1))
        q = double(2 * nc - 1);
    return int(q);
}

// Distinct cells c-1, c, c+1 (periodic) along one axis; fewer when the axis
// has fewer than three cells, so no cell is visited twice.
__device__ __forceinline__ int stencil_axis(int c, int nc, int out[3]) {
    if (nc >= 3) {
        out[0] = (c == 0) ? nc - 1 : c - 1;
        out[1] = c;
        out[2] = (c == nc - 1) ? 0 : c + 1;
        return 3;
    }
    out[0] = 0;
    out[1] = 1;
    return nc;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace tmd

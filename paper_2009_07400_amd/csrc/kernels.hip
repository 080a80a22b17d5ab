// HIP kernels for gfx950 (MI355X): cell binning, full neighbor-list build,
// Lennard-Jones force sum fused with the velocity-Verlet kicks and drift,
// deterministic reductions, and state load/unload.
//
// Method (tinyMD, arXiv 2009.07400): Lennard-Jones 12-6 force, Sec. 3.2 Eq. 2
// and the compute_potential example of Sec. 4.2; Verlet lists built from cell
// lists at cutoff + skin, Sec. 3.2 and Fig. 1; neighbor-major list layout for
// GPUs, Sec. 4.2; velocity Verlet of Newton's law (Sec. 3.2, Eq. 1) with the
// list rebuilt every `rebuild_every` steps (Sec. 6).
//
// Layout in HBM: positions, velocities and forces are structure-of-arrays
// FP64 in cell-sorted order; the list is int32, row k of the list holds the
// k-th neighbor of every atom (nbr[k * np + i]), so lane i of a wavefront
// reads a contiguous 256-byte segment per row.
#include "internal.h"

#include <math.h>

namespace tmd {

namespace {

// Workgroup index remapped so that the workgroups the hardware places on one
// XCD (b, b + 8, b + 16, ...) process one contiguous range of atoms.  Atoms
// are sorted by cell, so each XCD's L2 then holds one spatial slab of the box
// and the neighbor gathers of its workgroups hit that L2.
__device__ __forceinline__ int xcd_block() {
    const int b = blockIdx.x, nb = gridDim.x;  // nb is a multiple of kNumXcd
    return (b % kNumXcd) * (nb / kNumXcd) + b / kNumXcd;
}

// Minimum-image difference along one axis: d = a - b, shifted by one box
// length when |d| > L/2 (positions are kept in [0, L)).
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
// already is the minimum image.  The correction therefore sits behind a
// branch that a wavefront takes only when one of its lanes needs it, and it
// applies the same per-axis rule as mic(), so the result is bit-identical.
__device__ __forceinline__ double pair_delta(double xi, double yi, double zi, double xj, double yj, double zj,
                                            double L, double halfL, double &dx, double &dy, double &dz) {
    dx = xi - xj;
    dy = yi - yj;
    dz = zi - zj;
    const bool wrapped = int(fabs(dx) > halfL) | int(fabs(dy) > halfL) | int(fabs(dz) > halfL);
    if (wrapped) {
        dx = mic(dx, L, halfL);
        dy = mic(dy, L, halfL);
        dz = mic(dz, L, halfL);
    }
    return dist2(dx, dy, dz);
}

// 1/s for s > 0: hardware reciprocal estimate refined by two Newton-Raphson
// steps r <- r + r (1 - s r), which roughly squares the relative error each
// time; the result is within an ulp or two of the correctly rounded value.
__device__ __forceinline__ double recip(double s) {
    double r = __builtin_amdgcn_rcp(s);
    double e = fma(-s, r, 1.0);
    r = fma(r, e, r);
    e = fma(-s, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double wrap(double p, double L) {
    if (p >= L)
        p -= L;
    if (p < 0.0)
        p += L;
    return p;
}

__device__ __forceinline__ int cell_coord(double p, const Geom &g) {
    double q = floor(p / g.side);
    if (!(q >= 0.0))  // also catches NaN
        q = 0.0;
    if (q > double(g.nc - 1))
        q = double(g.nc - 1);
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

// Deterministic workgroup sum of three values; result valid in thread 0.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c) {
    __shared__ double red[3][kBlock / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = a;
        red[1][wave] = b;
        red[2][wave] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = b = c = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) {
            a += red[0][w];
            b += red[1][w];
            c += red[2][w];
        }
    }
}

// ------------------------------------------------------------------ utility

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_load_state(Geom g, const double *__restrict__ ix,
                                                       const double *__restrict__ iy, const double *__restrict__ iz,
                                                       const double *__restrict__ ivx, const double *__restrict__ ivy,
                                                       const double *__restrict__ ivz, double *x, double *y, double *z,
                                                       double *vx, double *vy, double *vz, int32_t *orig, int32_t *err) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n)
        return;
    const double px = wrap(ix[i], g.L), py = wrap(iy[i], g.L), pz = wrap(iz[i], g.L);
    const double a = ivx[i], b = ivy[i], c = ivz[i];
    if (!(isfinite(a) && isfinite(b) && isfinite(c)))
        atomicOr(err, kErrNonFinite);
    if (!(px >= 0.0 && px < g.L && py >= 0.0 && py < g.L && pz >= 0.0 && pz < g.L))
        atomicOr(err, isfinite(px) && isfinite(py) && isfinite(pz) ? kErrOutOfBox : kErrNonFinite);
    x[i] = px;
    y[i] = py;
    z[i] = pz;
    vx[i] = a;
    vy[i] = b;
    vz[i] = c;
    orig[i] = i;
}

__global__ __launch_bounds__(kBlock) void k_unload(int n, const double *__restrict__ ax, const double *__restrict__ ay,
                                                   const double *__restrict__ az, const int32_t *__restrict__ orig,
                                                   double *o0, double *o1, double *o2) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= n)
        return;
    const int o = orig[p];
    if (o0)
        o0[o] = ax[p];
    if (o1)
        o1[o] = ay[p];
    if (o2)
        o2[o] = az[p];
}

// ------------------------------------------------------------------ binning

// Cell of every atom and its arrival slot within the cell.
__global__ __launch_bounds__(kBlock) void k_bin_count(Geom g, const double *__restrict__ x,
                                                      const double *__restrict__ y, const double *__restrict__ z,
                                                      int32_t *cell_of, int32_t *slot, int32_t *cell_count,
                                                      int32_t *err) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n)
        return;
    const double px = x[i], py = y[i], pz = z[i];
    if (!(isfinite(px) && isfinite(py) && isfinite(pz)))
        atomicOr(err, kErrNonFinite);
    const int c = (cell_coord(pz, g) * g.nc + cell_coord(py, g)) * g.nc + cell_coord(px, g);
    cell_of[i] = c;
    slot[i] = atomicAdd(&cell_count[c], 1);
}

// Exclusive scan, level 1: each workgroup scans a tile of kScanTile counts
// (four per thread) and records the tile total.
__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                    int32_t *__restrict__ sums, int n) {
    __shared__ int32_t sh[256];
    const int t = threadIdx.x;
    const int base = blockIdx.x * kScanTile + t * 4;
    int v[4], tot = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = (base + q < n) ? in[base + q] : 0;
        tot += v[q];
    }
    sh[t] = tot;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int run = sh[t] - tot;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (base + q < n)
            out[base + q] = run;
        run += v[q];
    }
    if (t == 255)
        sums[blockIdx.x] = sh[255];
}

// Level 2: one workgroup turns the tile totals into exclusive offsets and
// writes the grand total to out[n].
__global__ __launch_bounds__(1024) void k_scan_sums(int32_t *sums, int nt, int32_t *out, int n) {
    __shared__ int32_t sh[1024];
    const int t = threadIdx.x;
    const int per = (nt + 1023) / 1024;
    const int b0 = t * per;
    int tot = 0;
    for (int q = 0; q < per; ++q)
        if (b0 + q < nt)
            tot += sums[b0 + q];
    sh[t] = tot;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int run = sh[t] - tot;
    for (int q = 0; q < per; ++q)
        if (b0 + q < nt) {
            const int v = sums[b0 + q];
            sums[b0 + q] = run;
            run += v;
        }
    if (t == 1023)
        out[n] = sh[1023];
}

__global__ __launch_bounds__(256) void k_scan_add(int32_t *out, const int32_t *__restrict__ sums, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        out[i] += sums[i / kScanTile];
}

__global__ __launch_bounds__(kBlock) void k_scatter(int n, const int32_t *__restrict__ cell_of,
                                                    const int32_t *__restrict__ slot,
                                                    const int32_t *__restrict__ cell_start, int32_t *tmp_idx) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        tmp_idx[cell_start[cell_of[i]] + slot[i]] = i;
}

// Atomic arrival order inside a cell is not reproducible; order each cell's
// members by original atom id so the whole pipeline is deterministic.
__global__ __launch_bounds__(kBlock) void k_cell_sort(int ncell, const int32_t *__restrict__ cell_start,
                                                      int32_t *tmp_idx, const int32_t *__restrict__ orig) {
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell)
        return;
    const int b = cell_start[c], e = cell_start[c + 1];
    for (int p = b + 1; p < e; ++p) {
        const int v = tmp_idx[p];
        const int key = orig[v];
        int q = p - 1;
        while (q >= b && orig[tmp_idx[q]] > key) {
            tmp_idx[q + 1] = tmp_idx[q];
            --q;
        }
        tmp_idx[q + 1] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_permute(int n, const int32_t *__restrict__ tmp_idx,
                                                    const double *__restrict__ x, const double *__restrict__ y,
                                                    const double *__restrict__ z, const double *__restrict__ vx,
                                                    const double *__restrict__ vy, const double *__restrict__ vz,
                                                    const int32_t *__restrict__ orig, double *x2, double *y2,
                                                    double *z2, double *vx2, double *vy2, double *vz2,
                                                    int32_t *orig2) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= n)
        return;
    const int p = tmp_idx[q];
    x2[q] = x[p];
    y2[q] = y[p];
    z2[q] = z[p];
    vx2[q] = vx[p];
    vy2[q] = vy[p];
    vz2[q] = vz[p];
    orig2[q] = orig[p];
}

// ------------------------------------------------------------------ neighbor list

// One lane per atom (cell-sorted order): scan the distinct cells of the
// 27-cell stencil and keep every j != i with s < (cutoff + skin)^2.
__global__ __launch_bounds__(kBlock) void k_build(Geom g, const double *__restrict__ x, const double *__restrict__ y,
                                                  const double *__restrict__ z,
                                                  const int32_t *__restrict__ cell_start, int32_t *__restrict__ cnt,
                                                  int32_t *__restrict__ nbr, int32_t *err) {
    const int i = xcd_block() * kBlock + threadIdx.x;
    if (i >= g.n)
        return;
    const double xi = x[i], yi = y[i], zi = z[i];
    int sx[3], sy[3], sz[3];
    const int nx = stencil_axis(cell_coord(xi, g), g.nc, sx);
    const int ny = stencil_axis(cell_coord(yi, g), g.nc, sy);
    const int nz = stencil_axis(cell_coord(zi, g), g.nc, sz);
    int c = 0;
    for (int a = 0; a < nz; ++a)
        for (int b = 0; b < ny; ++b)
            for (int d = 0; d < nx; ++d) {
                const int cell = (sz[a] * g.nc + sy[b]) * g.nc + sx[d];
                const int e = cell_start[cell + 1];
                for (int p = cell_start[cell]; p < e; ++p) {
                    if (p == i)
                        continue;
                    double dx, dy, dz;
                    if (pair_delta(xi, yi, zi, x[p], y[p], z[p], g.L, g.halfL, dx, dy, dz) < g.rl2) {
                        if (c < g.maxnb)
                            nbr[int64_t(c) * g.np + i] = p;
                        ++c;
                    }
                }
            }
    cnt[i] = c < g.maxnb ? c : g.maxnb;
    if (c > g.maxnb) {
        atomicOr(err, kErrOverflow);
        atomicMax(err + 1, c);
    }
}

// ------------------------------------------------------------------ force

// One lane per atom: F_i = sum over the list of f(s) d_ij for s < cutoff^2
// with f = 48 eps sr6 (sr6 - 1/2) sr2, sr2 = 1/s, sr6 = sigma^6 sr2^3.
// MODE 0: store F.  MODE 1: store F, kick v += h F.  MODE 2: kick twice
// (closing this step and opening the next) and drift into the other buffer.
// With THERMO, each workgroup writes its partial sums of the pair energy,
// of s f(s) and of |v|^2 (the full-step velocity) - no atomics anywhere.
template <int MODE, bool THERMO>
__global__ __launch_bounds__(kBlock) void k_force(Geom g, const double *__restrict__ x, const double *__restrict__ y,
                                                  const double *__restrict__ z, const int32_t *__restrict__ cnt,
                                                  const int32_t *__restrict__ nbr, double *__restrict__ vx,
                                                  double *__restrict__ vy, double *__restrict__ vz,
                                                  double *__restrict__ fx, double *__restrict__ fy,
                                                  double *__restrict__ fz, double *__restrict__ xo,
                                                  double *__restrict__ yo, double *__restrict__ zo,
                                                  double *__restrict__ partials, int32_t *err) {
    const int blk = xcd_block();
    const int i = blk * kBlock + threadIdx.x;
    double u = 0.0, w = 0.0, ke = 0.0;
    if (i < g.n) {
        const double xi = x[i], yi = y[i], zi = z[i];
        double ax = 0.0, ay = 0.0, az = 0.0;
        const int c = cnt[i];
        const int32_t *row = nbr + i;
        // Two-stage pipeline: the positions of pair k+1 and the index of
        // pair k+2 are in flight while pair k is evaluated.  The index stream
        // is read once per step, so it is loaded non-temporally and leaves
        // the caches to the position gathers.
        int jn = (c > 1) ? __builtin_nontemporal_load(row + g.np) : i;
        int j0 = (c > 0) ? __builtin_nontemporal_load(row) : i;
        double xj = x[j0], yj = y[j0], zj = z[j0];
        for (int k = 0; k < c; ++k) {
            const double xc = xj, yc = yj, zc = zj;
            if (k + 1 < c) {
                xj = x[jn];
                yj = y[jn];
                zj = z[jn];
                jn = (k + 2 < c) ? __builtin_nontemporal_load(row + int64_t(k + 2) * g.np) : i;
            }
            double dx, dy, dz;
            const double s = pair_delta(xi, yi, zi, xc, yc, zc, g.L, g.halfL, dx, dy, dz);
            if (s < g.rc2) {
                const double sr2 = recip(s);
                const double sr6 = sr2 * sr2 * sr2 * g.sigma6;
                const double f = 48.0 * sr6 * (sr6 - 0.5) * sr2 * g.eps;
                ax += f * dx;
                ay += f * dy;
                az += f * dz;
                if (THERMO) {
                    u += 4.0 * g.eps * (sr6 * sr6 - sr6);
                    w += s * f;
                }
            }
        }
        if (MODE == 0 || MODE == 1) {
            fx[i] = ax;
            fy[i] = ay;
            fz[i] = az;
            if (!(isfinite(ax) && isfinite(ay) && isfinite(az)))
                atomicOr(err, kErrNonFinite);
        }
        if (MODE >= 1) {
            double a = vx[i] + g.h * ax, b = vy[i] + g.h * ay, d = vz[i] + g.h * az;
            if (THERMO)
                ke = a * a + b * b + d * d;
            if (MODE == 2) {
                a = a + g.h * ax;
                b = b + g.h * ay;
                d = d + g.h * az;
                const double nx = wrap(xi + g.dt * a, g.L), ny = wrap(yi + g.dt * b, g.L),
                             nz = wrap(zi + g.dt * d, g.L);
                xo[i] = nx;
                yo[i] = ny;
                zo[i] = nz;
                if (!(isfinite(nx) && isfinite(ny) && isfinite(nz)))
                    atomicOr(err, kErrNonFinite);
            }
            vx[i] = a;
            vy[i] = b;
            vz[i] = d;
        }
    }
    if (THERMO) {
        block_sum3(u, w, ke);
        if (threadIdx.x == 0) {
            partials[blk * kPartialStride + 0] = u;
            partials[blk * kPartialStride + 1] = w;
            partials[blk * kPartialStride + 2] = ke;
        }
    }
}

// First half of a step when F of the current positions is already stored.
__global__ __launch_bounds__(kBlock) void k_drift(Geom g, const double *__restrict__ x, const double *__restrict__ y,
                                                  const double *__restrict__ z, double *__restrict__ vx,
                                                  double *__restrict__ vy, double *__restrict__ vz,
                                                  const double *__restrict__ fx, const double *__restrict__ fy,
                                                  const double *__restrict__ fz, double *__restrict__ xo,
                                                  double *__restrict__ yo, double *__restrict__ zo, int32_t *err) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n)
        return;
    const double a = vx[i] + g.h * fx[i], b = vy[i] + g.h * fy[i], d = vz[i] + g.h * fz[i];
    vx[i] = a;
    vy[i] = b;
    vz[i] = d;
    const double nx = wrap(x[i] + g.dt * a, g.L), ny = wrap(y[i] + g.dt * b, g.L), nz = wrap(z[i] + g.dt * d, g.L);
    xo[i] = nx;
    yo[i] = ny;
    zo[i] = nz;
    if (!(isfinite(nx) && isfinite(ny) && isfinite(nz)))
        atomicOr(err, kErrNonFinite);
}

// Sum the per-workgroup partials in a fixed order (one workgroup).
__global__ __launch_bounds__(kBlock) void k_reduce(Geom g, const double *__restrict__ partials, int nblk,
                                                   double *out, int row_len) {
    double u = 0.0, w = 0.0, k = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBlock) {
        u += partials[b * kPartialStride + 0];
        w += partials[b * kPartialStride + 1];
        k += partials[b * kPartialStride + 2];
    }
    block_sum3(u, w, k);
    if (threadIdx.x == 0) {
        const double U = 0.5 * u, W = 0.5 * w, KE = 0.5 * g.mass * k;
        if (row_len == 2) {
            out[0] = U;
            out[1] = W;
        } else {
            out[0] = KE;
            out[1] = g.n > 1 ? 2.0 * KE / (3.0 * g.n - 3.0) : 0.0;
            out[2] = U;
            out[3] = W;
            out[4] = KE + U;
        }
    }
}

// Current list in original ids, each row sorted ascending, unused slots -1.
__global__ __launch_bounds__(kBlock) void k_export_neighbors(Geom g, const int32_t *__restrict__ cnt,
                                                             const int32_t *__restrict__ nbr,
                                                             const int32_t *__restrict__ orig, int32_t *counts,
                                                             int32_t *ids) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= g.n)
        return;
    const int o = orig[p], c = cnt[p];
    int32_t *row = ids + int64_t(o) * g.maxnb;
    for (int k = 0; k < c; ++k) {
        const int v = orig[nbr[int64_t(k) * g.np + p]];
        int q = k - 1;
        while (q >= 0 && row[q] > v) {
            row[q + 1] = row[q];
            --q;
        }
        row[q + 1] = v;
    }
    for (int k = c; k < g.maxnb; ++k)
        row[k] = -1;
    counts[o] = c;
}

inline int blocks_for(int64_t n, int b) { return int((n + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0)
        return hipSuccess;
    k_fill_i32<<<blocks_for(n, 256), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_load_state(const Geom &g, const double *const pos[3], const double *const vel[3], Buffers &b,
                             Cursor c, hipStream_t s) {
    k_load_state<<<blocks_for(g.n, kBlock), kBlock, 0, s>>>(g, pos[0], pos[1], pos[2], vel[0], vel[1], vel[2],
                                                            b.x[c.x], b.y[c.x], b.z[c.x], b.vx[c.o], b.vy[c.o],
                                                            b.vz[c.o], b.orig[c.o], b.err);
    return hipGetLastError();
}

hipError_t launch_unload(const Geom &g, const double *ax, const double *ay, const double *az, const int32_t *orig,
                         double *const out[3], hipStream_t s) {
    k_unload<<<blocks_for(g.n, kBlock), kBlock, 0, s>>>(g.n, ax, ay, az, orig, out[0], out[1], out[2]);
    return hipGetLastError();
}

hipError_t launch_bin(const Geom &g, Buffers &b, Cursor c, hipStream_t s) {
    const int cur = c.x, nxt = 1 - c.x, o = c.o, on = 1 - c.o;
    hipError_t e = launch_fill_i32(b.cell_count, 0, g.ncell, s);
    if (e != hipSuccess)
        return e;
    k_bin_count<<<blocks_for(g.n, kBlock), kBlock, 0, s>>>(g, b.x[cur], b.y[cur], b.z[cur], b.cell_of, b.slot,
                                                           b.cell_count, b.err);
    const int nt = scan_blocks(g.ncell);
    k_scan_tiles<<<nt, 256, 0, s>>>(b.cell_count, b.cell_start, b.scan_sums, g.ncell);
    k_scan_sums<<<1, 1024, 0, s>>>(b.scan_sums, nt, b.cell_start, g.ncell);
    k_scan_add<<<blocks_for(g.ncell, 256), 256, 0, s>>>(b.cell_start, b.scan_sums, g.ncell);
    k_scatter<<<blocks_for(g.n, kBlock), kBlock, 0, s>>>(g.n, b.cell_of, b.slot, b.cell_start, b.tmp_idx);
    k_cell_sort<<<blocks_for(g.ncell, kBlock), kBlock, 0, s>>>(g.ncell, b.cell_start, b.tmp_idx, b.orig[o]);
    k_permute<<<blocks_for(g.n, kBlock), kBlock, 0, s>>>(g.n, b.tmp_idx, b.x[cur], b.y[cur], b.z[cur], b.vx[o],
                                                         b.vy[o], b.vz[o], b.orig[o], b.x[nxt], b.y[nxt],
                                                         b.z[nxt], b.vx[on], b.vy[on], b.vz[on], b.orig[on]);
    return hipGetLastError();
}

hipError_t launch_build(const Geom &g, Buffers &b, Cursor c, hipStream_t s) {
    k_build<<<atom_grid(g.n), kBlock, 0, s>>>(g, b.x[c.x], b.y[c.x], b.z[c.x], b.cell_start, b.nbr_count, b.nbr,
                                              b.err);
    return hipGetLastError();
}

template <int MODE, bool THERMO>
static void force_variant(const Geom &g, Buffers &b, Cursor c, hipStream_t s) {
    const int cur = c.x, nxt = 1 - c.x;
    k_force<MODE, THERMO><<<atom_grid(g.n), kBlock, 0, s>>>(
        g, b.x[cur], b.y[cur], b.z[cur], b.nbr_count, b.nbr, b.vx[c.o], b.vy[c.o], b.vz[c.o], b.fx, b.fy, b.fz,
        b.x[nxt], b.y[nxt], b.z[nxt], b.partials, b.err);
}

hipError_t launch_force(const Geom &g, Buffers &b, Cursor cur, int mode, bool thermo, hipStream_t s) {
    switch (mode * 2 + (thermo ? 1 : 0)) {
    case 0: force_variant<0, false>(g, b, cur, s); break;
    case 1: force_variant<0, true>(g, b, cur, s); break;
    case 2: force_variant<1, false>(g, b, cur, s); break;
    case 3: force_variant<1, true>(g, b, cur, s); break;
    case 4: force_variant<2, false>(g, b, cur, s); break;
    case 5: force_variant<2, true>(g, b, cur, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_drift(const Geom &g, Buffers &b, Cursor c, hipStream_t s) {
    const int cur = c.x, nxt = 1 - c.x;
    k_drift<<<blocks_for(g.n, kBlock), kBlock, 0, s>>>(g, b.x[cur], b.y[cur], b.z[cur], b.vx[c.o], b.vy[c.o],
                                                       b.vz[c.o], b.fx, b.fy, b.fz, b.x[nxt], b.y[nxt], b.z[nxt],
                                                       b.err);
    return hipGetLastError();
}

hipError_t launch_reduce(const Geom &g, const Buffers &b, double *out, int row_len, hipStream_t s) {
    k_reduce<<<1, kBlock, 0, s>>>(g, b.partials, atom_grid(g.n), out, row_len);
    return hipGetLastError();
}

hipError_t launch_export_neighbors(const Geom &g, const Buffers &b, Cursor c, int32_t *counts, int32_t *ids,
                                   hipStream_t s) {
    k_export_neighbors<<<blocks_for(g.n, kBlock), kBlock, 0, s>>>(g, b.nbr_count, b.nbr, b.orig[c.o], counts, ids);
    return hipGetLastError();
}

}  // namespace tmd

// HIP kernels for gfx950 (MI355X): cell binning, neighbor-list build (full
// lists, or half lists inside blocks), the Lennard-Jones and Spring-Dashpot
// force sums fused with the velocity-Verlet kicks and drift, the adjoint's
// Hessian-vector product, deterministic per-box reductions, state load and
// unload, position layout conversion and list export, for one or many
// independent periodic boxes.
//
// Method (tinyMD, arXiv 2009.07400): LJ 12-6 force, Sec. 3.2 Eq. 2 and the
// compute_potential example of Sec. 4.2; Spring-Dashpot contact force, Sec.
// 3.2 Eq. 3; Verlet lists built from cell lists at cutoff + skin, Sec. 3.2
// and Fig. 1 (half lists and the subtracted partner force, Sec. 3.2 and the
// half_nb variant of Sec. 4.2); the particle layouts of Sec. 4.2; velocity
// Verlet of Newton's law (Sec. 3.2, Eq. 1) with the list rebuilt every
// `rebuild_every` steps (Sec. 6).
//
// Work decomposition.  Cells have side >= cutoff + skin.  Each box is cut
// into blocks of E x E x E cells (E = 2 or 3; a small box is one block) and
// atoms are stored block-major, so the atoms of a block, and of each of its
// cells, are contiguous.  One workgroup owns one block: it copies the
// positions of the block's neighborhood (the (E+2)^3 cells around it, fewer
// in small boxes) into LDS, and its lanes - one to four per atom - gather
// neighbor positions from LDS instead of from the L2.  The list stores LDS
// slot numbers (16 bits) for such blocks; a block whose neighborhood exceeds
// the LDS capacity gathers from global memory and its list stores global
// atom indices (32 bits).
//
// Layout in HBM: velocities and forces are structure-of-arrays FP64,
// positions SoA, AoS or AoSoA (PosL); the list is tiled neighbor-major (64
// atoms per tile, rows of 16 bytes per atom), so a wavefront reads one
// contiguous 1 KB row per load.
#include <math.h>

#include "device.h"
#include "internal.h"

namespace tmd {

namespace {

// Workgroup index remapped so that the workgroups the hardware places on one
// XCD (b, b + 8, b + 16, ...) process one contiguous range of blocks, i.e.
// one spatial slab of a box, which then stays in that XCD's L2.
__device__ __forceinline__ int xcd_remap() {
    const int b = blockIdx.x, nb = gridDim.x;  // nb is a multiple of kNumXcd
    return (b % kNumXcd) * (nb / kNumXcd) + b / kNumXcd;
}

// Workgroup -> (block, part): d.parts workgroups share one block, each taking
// a contiguous share of its atoms (and staging the whole neighborhood).
__device__ __forceinline__ bool block_part(const Dims &d, int &b, int &part) {
    const int wg = xcd_remap();
    b = wg >> (d.parts >> 1);  // parts is 1, 2 or 4
    part = wg & (d.parts - 1);
    return b < d.nblk;
}

// Block coordinate and offset inside the block of cell coordinate c.
__device__ __forceinline__ void split_edge(int c, int E, int &blk, int &loc) {
    blk = (E == 2) ? (c >> 1) : (c / E);
    loc = c - blk * E;
}

__device__ __forceinline__ int cell_slot(const Box &B, int cx, int cy, int cz) {
    const int E = B.edge;
    int bx, lx, by, ly, bz, lz;
    split_edge(cx, E, bx, lx);
    split_edge(cy, E, by, ly);
    split_edge(cz, E, bz, lz);
    const int blk = (bz * B.nbx + by) * B.nbx + bx;
    return B.cell_off + blk * (E * E * E) + (lz * E + ly) * E + lx;
}

constexpr int kAxis = kMaxEdge + 2;  // neighborhood cells per axis, at most

// Distinct cells c0-1 .. c0+e (periodic) along one axis, in that order.
__device__ __forceinline__ int hood_axis(int c0, int e, int nc, int out[kAxis]) {
    int n = 0;
    for (int t = 0; t < e + 2; ++t) {
        int v = c0 - 1 + t;
        v = v < 0 ? v + nc : (v >= nc ? v - nc : v);
        bool dup = false;
        for (int q = 0; q < n; ++q)
            dup |= (out[q] == v);
        if (!dup)
            out[n++] = v;
    }
    return n;
}

// Neighborhood axes of local block lb (uniform across the workgroup).
__device__ __forceinline__ void hood_axes(const Box &B, int lb, int n[3], int co[3][kAxis]) {
    const int nbx = B.nbx;
    const int bc[3] = {lb % nbx, (lb / nbx) % nbx, lb / (nbx * nbx)};
    for (int a = 0; a < 3; ++a) {
        const int c0 = B.edge * bc[a];
        const int e = min(B.edge, B.nc - c0);
        n[a] = hood_axis(c0, e, B.nc, co[a]);
    }
}

struct Hood {
    int cs[kMaxHood];       // first atom of each neighborhood cell
    int off[kMaxHood + 1];  // LDS slot of each cell's first atom; off[ncell] = atoms staged
    int ncell;
    int a0, a1;             // the block's own atoms

    // the atoms of share `part` of `parts`
    __device__ __forceinline__ void share(int part, int parts, int &lo, int &hi) const {
        const int n = a1 - a0;
        lo = a0 + (n * part) / parts;
        hi = a0 + (n * (part + 1)) / parts;
    }
};

__device__ __forceinline__ int wave_prefix_incl(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o)
            v += t;
    }
    return v;
}

// Cell ranges and LDS offsets of the neighborhood of local block lb (the
// first wavefront handles cells u and u + 64); ends with a workgroup barrier.
__device__ __forceinline__ void hood_setup(const Box &B, int lb, const int32_t *__restrict__ cell_start, Hood &h) {
    if (threadIdx.x < 64) {
        int n[3], co[3][kAxis];
        hood_axes(B, lb, n, co);
        const int nh = n[0] * n[1] * n[2];
        // all cell_start reads first (one memory round trip, the block's own
        // atom range included), then the scans
        const int cpb = B.edge * B.edge * B.edge;
        const int first = B.cell_off + lb * cpb;
        int a01[2] = {0, 0};
        if (threadIdx.x == 0) {
            a01[0] = cell_start[first * kSub];
            a01[1] = cell_start[(first + cpb) * kSub];
        }
        int cs[2] = {0, 0}, cnt[2] = {0, 0};
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int u = threadIdx.x + 64 * half;
            if (u < nh) {
                const int ix = u % n[0], iy = (u / n[0]) % n[1], iz = u / (n[0] * n[1]);
                const int sl = cell_slot(B, co[0][ix], co[1][iy], co[2][iz]) * kSub;
                cs[half] = cell_start[sl];
                cnt[half] = cell_start[sl + kSub];
            }
        }
        int base = 0;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int u = threadIdx.x + 64 * half;
            const int incl = base + wave_prefix_incl(cnt[half] - cs[half]);
            if (u < nh) {
                h.cs[u] = cs[half];
                h.off[u + 1] = incl;
            }
            base = __shfl(incl, 63, 64);
        }
        if (threadIdx.x == 0) {
            h.off[0] = 0;
            h.ncell = nh;
            h.a0 = a01[0];
            h.a1 = a01[1];
        }
    }
    __syncthreads();
}

static_assert(sizeof(Hood) <= kHoodWords * 4, "neighborhood table");

// The force kernel's dynamic LDS after the neighborhood copy: the table
// (rounded up to whole doubles), then block_sum3's scratch.
constexpr int kHoodBytes8 = int((sizeof(Hood) + 7) / 8 * 8);
static_assert(kHoodBytes8 + 3 * (kMaxThreads / 64) * 8 <= kForceLdsTail, "force kernel LDS tail");

// The list build stores each block's table (hood_setup's result) in HBM; the
// kernels that run on that list read it back in one coalesced round trip
// instead of recomputing it from cell_start.  Ends with a workgroup barrier.
__device__ __forceinline__ void hood_store(const Hood &h, int b, int32_t *__restrict__ tab) {
    const int *src = reinterpret_cast<const int *>(&h);
    for (int t = threadIdx.x; t < int(sizeof(Hood) / 4); t += blockDim.x)
        tab[int64_t(b) * kHoodWords + t] = src[t];
}

// The stored table read in two halves: hood_fetch() issues the global loads
// into registers (at least 64 threads, so four words each cover it), and
// hood_commit() writes them to LDS and ends with a workgroup barrier.  Loads
// issued in between (the box descriptor) share the table's round trip.
struct HoodWords {
    int v[kHoodWords / 64];
};

__device__ __forceinline__ void hood_fetch(const int32_t *__restrict__ tab, int b, HoodWords &w) {
    constexpr int n = int(sizeof(Hood) / 4);
    const int32_t *src = tab + int64_t(b) * kHoodWords;
#pragma unroll
    for (int k = 0; k < kHoodWords / 64; ++k) {
        const int t = threadIdx.x + k * int(blockDim.x);
        w.v[k] = t < n ? src[t] : 0;
    }
}

__device__ __forceinline__ void hood_commit(const HoodWords &w, Hood &h) {
    constexpr int n = int(sizeof(Hood) / 4);
    int *dst = reinterpret_cast<int *>(&h);
#pragma unroll
    for (int k = 0; k < kHoodWords / 64; ++k) {
        const int t = threadIdx.x + k * int(blockDim.x);
        if (t < n)
            dst[t] = w.v[k];
    }
    __syncthreads();
}

// Neighborhood cell holding LDS slot t (largest u with off[u] <= t).
__device__ __forceinline__ int hood_find(const Hood &h, int t) {
    int lo = 0, hi = h.ncell;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (h.off[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// hood_find for R slots at once: a fixed seven-step branchless search
// (kMaxHood < 128) whose R table reads per step are independent, so a thread
// waits for seven LDS round trips instead of seven per slot.  off[ncell]
// exceeds every slot, so probes past the last cell read it and never move.
template <int R>
__device__ __forceinline__ void hood_find_n(const Hood &h, const int (&t)[R], int (&u)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r)
        u[r] = 0;
#pragma unroll
    for (int step = 64; step > 0; step >>= 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int m = min(u[r] + step, h.ncell);
            u[r] = h.off[m] <= t[r] ? m : u[r];
        }
    }
}

// LDS copy of a neighborhood: packed (x, y, z) triples, 24 bytes per slot,
// addressed with 32-bit LDS pointers (one 24-bit multiply or multiply-add
// per atom, then reads with immediate offsets).
typedef __attribute__((address_space(3))) double lds_double;
typedef __attribute__((address_space(3))) char lds_char;

__device__ __forceinline__ lds_double *lds_slot(lds_double *base, int slot) {
    return (lds_double *)((lds_char *)base + __umul24(unsigned(slot), 24u));
}

struct GlobalPos {
    PosL P;
    __device__ __forceinline__ void get(int j, double &a, double &b, double &c) const { P.get(j, a, b, c); }
};

// Atom i of position buffer p in layout `lay`, for kernels that take the
// buffer as a restrict-qualified argument (so that its reads may move past
// the kernel's stores).  A kernel may pass its layout as a template
// constant: the list build does.
__device__ __forceinline__ void pos_get(int lay, int ntp, const double *__restrict__ p, int i, double &a, double &b,
                                        double &c) {
    PosL{const_cast<double *>(p), ntp, lay}.get(i, a, b, c);
}

__device__ __forceinline__ void pos_put(int lay, int ntp, double *__restrict__ p, int i, double a, double b,
                                        double c) {
    PosL{p, ntp, lay}.put(i, a, b, c);
}

__device__ __forceinline__ PosL pos_of(int lay, int ntp, const double *p) {
    return PosL{const_cast<double *>(p), ntp, lay};
}

// Periodic images of a neighborhood copy (the role of the shifted ghost
// copies of Sec. 4.3).  With `on`, every staged position is moved to its
// image nearest to the block's center (nearest_image()), so
// that for every atom of the block each list partner's copy is its image
// nearest to that atom and the pair loops take plain differences (no
// minimum-image test per pair).  `on` needs at least E + 3 cells per axis;
// below E + 4 (`check`) the pair loops also test each difference against
// L/2 (pair_geom).  The list build stages without images, as its neighbor
// decisions take the minimum image of the raw difference.
// Half lists (Sec. 3.2: each pair listed once, the partner taking the
// opposite force; the half_nb variant of Sec. 4.2) inside one block: a pair
// of two atoms of the block is listed once, by the atom with the lower LDS
// slot, and the force kernel adds the partner's reaction to a sum in LDS; a
// pair that crosses blocks is listed from both sides, each block computing
// its own atom's force, so no workgroup writes another's atoms.  The own
// cells sit at neighborhood coordinates 1..e per axis when the neighborhood
// holds no cell twice; their LDS slots then lie in [off[first own cell],
// off[last own cell + 1]), the span the reaction sums cover.
struct OwnCells {
    int e[3], n[3];  // own cells and neighborhood cells per axis
};

__device__ __forceinline__ bool own_cells(const Box &B, int lb, OwnCells &o) {
    const int nbx = B.nbx;
    const int bc[3] = {lb % nbx, (lb / nbx) % nbx, lb / (nbx * nbx)};
    bool plain = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        o.e[a] = min(B.edge, B.nc - B.edge * bc[a]);
        o.n[a] = o.e[a] + 2;
        plain &= B.nc >= o.n[a];
    }
    return plain;
}

// Whether block lb uses half lists, with its span's first slot and length:
// the system asks for them, one workgroup takes the whole block, its
// neighborhood is staged in LDS, holds no cell twice, and the span fits the
// reaction sums.  The list build and the force kernel decide alike from the
// same neighborhood table.
__device__ __forceinline__ bool block_half(const Dims &d, const Box &B, int lb, const Hood &h, bool fits, int &s_lo,
                                          int &span) {
    s_lo = span = 0;
    OwnCells o;
    if (!d.half || d.parts != 1 || !fits || !own_cells(B, lb, o))
        return false;
    const int ulo = (o.n[1] + 1) * o.n[0] + 1;
    const int uhi = (o.e[2] * o.n[1] + o.e[1]) * o.n[0] + o.e[0];
    s_lo = h.off[ulo];
    span = h.off[uhi + 1] - s_lo;
    return span <= d.rcap;
}

// LDS slot of the block's own atom i (global index) in a half-list block:
// the own cells in global order are those of compact index k over (lz, ly,
// lx), at neighborhood index ((lz + 1) n1 + ly + 1) n0 + lx + 1; i lies in
// the last of them that starts at or before it.
__device__ __forceinline__ int own_slot(const Box &B, int lb, const Hood &h, int i) {
    OwnCells o;
    own_cells(B, lb, o);
    const int nown = o.e[0] * o.e[1] * o.e[2];
    auto uo = [&](int k) {
        const int lx = k % o.e[0], r = k / o.e[0], ly = r % o.e[1], lz = r / o.e[1];
        return ((lz + 1) * o.n[1] + ly + 1) * o.n[0] + lx + 1;
    };
    int k = 0;
#pragma unroll
    for (int st = 16; st > 0; st >>= 1) {  // nown <= 27
        const int m = k + st;
        if (m < nown && h.cs[uo(m)] <= i)
            k = m;
    }
    const int u = uo(k);
    return h.off[u] + (i - h.cs[u]);
}

struct HoodImage {
    bool on;     // the neighborhood is staged at images near the block
    bool check;  // ... and a pair may still need its minimum image (pair_geom<2>)
    double cx, cy, cz, L, halfL;
};

__device__ __forceinline__ HoodImage hood_image(const Box &B, int lb, bool want) {
    HoodImage m;
    m.on = want && B.nc >= B.edge + 3;
    m.check = B.nc < B.edge + 4;
    const int nbx = B.nbx;
    const int bc[3] = {lb % nbx, (lb / nbx) % nbx, lb / (nbx * nbx)};
    double c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int c0 = B.edge * bc[a];
        const int e = min(B.edge, B.nc - c0);
        c[a] = (double(c0) + 0.5 * double(e)) * B.side;
    }
    m.cx = c[0];
    m.cy = c[1];
    m.cz = c[2];
    m.L = B.L;
    m.halfL = B.halfL;
    return m;
}

// Pair difference and |d|^2 for the block kernels' pair loops: IMG 0 takes
// the minimum image per pair (pair_delta_fma); IMG 1 the staged image
// (pair_delta_img), which is the image nearest to i when the box has at
// least E + 4 cells per axis; IMG 2 the staged image for boxes of E + 3
// cells, where it is the nearest one unless the pair's atoms moved more
// than (3 a / 2 - cutoff - skin) / 3 since the list build.  A wrong image
// puts the difference at least L/2 from zero along an axis, so such a
// pair fails |d|^2 < (L/2)^2 and its difference then takes the minimum
// image along each axis - the value of the other paths up to the rounding
// of one more subtraction of L.  With the right images all three give the
// same bits.
template <int IMG>
__device__ __forceinline__ double pair_geom(double xi, double yi, double zi, double xj, double yj, double zj,
                                            const Box &B, double &dx, double &dy, double &dz) {
    if (IMG == 0)
        return pair_delta_fma(xi, yi, zi, xj, yj, zj, B.L, B.invL, dx, dy, dz);
    double s = pair_delta_img(xi, yi, zi, xj, yj, zj, dx, dy, dz);
    if (IMG == 2 && s >= B.halfL2) {
        dx = mic(dx, B.L, B.halfL);
        dy = mic(dy, B.L, B.halfL);
        dz = mic(dz, B.L, B.halfL);
        s = fma(dz, dz, fma(dy, dy, dx * dx));
    }
    return s;
}

// Copy the neighborhood's positions into LDS (the global loads are
// coalesced within each cell), and a NaN sentinel atom at slot `sent` (the
// LDS capacity, the same slot for every block): list padding points there,
// and every comparison with a NaN distance is false, so padded entries need
// no test.  Ends with a workgroup barrier.
__device__ __forceinline__ void hood_stage(const Hood &h, int total, int sent, const PosL &P, lds_double *s,
                                           const HoodImage &im) {
    // four slots per thread per round: the four searches, then all twelve
    // global loads in flight together, then the LDS writes.  Every memory
    // operation is unconditional: a slot past the end copies the last atom
    // into the scratch slot after the sentinel.
    constexpr int R = 4;
    const int T = blockDim.x;
    for (int base = threadIdx.x; base < total; base += R * T) {
        int ts[R], us[R], g[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            ts[r] = min(base + r * T, total - 1);
        hood_find_n<R>(h, ts, us);
#pragma unroll
        for (int r = 0; r < R; ++r)
            g[r] = h.cs[us[r]] + (ts[r] - h.off[us[r]]);
        double px[R], py[R], pz[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            P.get(g[r], px[r], py[r], pz[r]);
        if (im.on) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                px[r] = nearest_image(px[r], im.cx, im.L, im.halfL);
                py[r] = nearest_image(py[r], im.cy, im.L, im.halfL);
                pz[r] = nearest_image(pz[r], im.cz, im.L, im.halfL);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            lds_double *a = lds_slot(s, base + r * T < total ? base + r * T : sent + 1);
            a[0] = px[r];
            a[1] = py[r];
            a[2] = pz[r];
        }
    }
    if (threadIdx.x == 0) {
        const double nan = __builtin_nan("");
        lds_double *a = lds_slot(s, sent);
        a[0] = nan;
        a[1] = nan;
        a[2] = nan;
    }
    __syncthreads();
}

// Deterministic workgroup sum of three values; valid in thread 0.  red is
// LDS scratch of 3 * kMaxThreads / 64 doubles.
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double (*red)[kMaxThreads / 64]) {
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
        for (int w = 0; w < int(blockDim.x >> 6); ++w) {
            a += red[0][w];
            b += red[1][w];
            c += red[2][w];
        }
    }
}

__device__ __forceinline__ void block_sum3(double &a, double &b, double &c) {
    __shared__ double red[3][kMaxThreads / 64];
    block_sum3(a, b, c, red);
}

// ------------------------------------------------------------------ utility

// NaN sentinel atom at slot nt of position buffers 1..count of a
// trajectory store (buffer j holds x, y, z at stride np from
// traj + 3 j np): 32-bit list padding points there.
__global__ void k_traj_sentinels(double *traj, int64_t np, int nt, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 3 * count)
        traj[(int64_t(t / 3 + 1) * 3 + t % 3) * np + nt] = __builtin_nan("");
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

__global__ __launch_bounds__(kAtomThreads) void k_load_state(Dims d, const Box *__restrict__ boxes,
                                                             const int32_t *__restrict__ atom_box,
                                                             const double *__restrict__ ix,
                                                             const double *__restrict__ iy,
                                                             const double *__restrict__ iz,
                                                             const double *__restrict__ ivx,
                                                             const double *__restrict__ ivy,
                                                             const double *__restrict__ ivz, PosL P, double *vx,
                                                             double *vy, double *vz, int32_t *orig, PosL P2,
                                                             int32_t *err) {
    const int i = blockIdx.x * kAtomThreads + threadIdx.x;
    if (i == 0) {
        // sentinel atom at slot nt of both position buffers: list padding of
        // blocks that gather from global memory points here
        const double nan = __builtin_nan("");
        P.put(d.nt, nan, nan, nan);
        P2.put(d.nt, nan, nan, nan);
    }
    if (i >= d.nt)
        return;
    const double L = boxes[atom_box[i]].L;
    const double px = wrap(ix[i], L), py = wrap(iy[i], L), pz = wrap(iz[i], L);
    const double a = ivx ? ivx[i] : 0.0, b = ivy ? ivy[i] : 0.0, c = ivz ? ivz[i] : 0.0;
    if (!(isfinite(a) && isfinite(b) && isfinite(c)))
        atomicOr(err, kErrNonFinite);
    if (!(px >= 0.0 && px < L && py >= 0.0 && py < L && pz >= 0.0 && pz < L))
        atomicOr(err, isfinite(px) && isfinite(py) && isfinite(pz) ? kErrOutOfBox : kErrNonFinite);
    P.put(i, px, py, pz);
    vx[i] = a;
    vy[i] = b;
    vz[i] = c;
    orig[i] = i;
}

// Scatter per-atom vectors back to original order.
__global__ __launch_bounds__(kAtomThreads) void k_unload(int n, const double *__restrict__ ax,
                                                         const double *__restrict__ ay,
                                                         const double *__restrict__ az,
                                                         const int32_t *__restrict__ orig, double *o0, double *o1,
                                                         double *o2) {
    const int p = blockIdx.x * kAtomThreads + threadIdx.x;
    if (p >= n)
        return;
    const int o = orig[p];
    const double a = ax[p], b = ay[p], c = az[p];
    if (o0)
        o0[o] = a;
    if (o1)
        o1[o] = b;
    if (o2)
        o2[o] = c;
}

// Positions back to original order, wrapped into [0, L) on the way (they
// drift unwrapped between list builds).
__global__ __launch_bounds__(kAtomThreads) void k_unload_pos(int n, PosL P, const int32_t *__restrict__ orig,
                                                             double *o0, double *o1, double *o2,
                                                             const Box *__restrict__ boxes,
                                                             const int32_t *__restrict__ atom_box) {
    const int p = blockIdx.x * kAtomThreads + threadIdx.x;
    if (p >= n)
        return;
    const int o = orig[p];
    double a, b, c;
    P.get(p, a, b, c);
    const double L = boxes[atom_box[p]].L;
    o0[o] = wrap(a, L);
    o1[o] = wrap(b, L);
    o2[o] = wrap(c, L);
}

// Copy a position buffer (all ntp slots, the sentinel included) into
// another buffer in another layout.
__global__ __launch_bounds__(kAtomThreads) void k_relayout(int ntp, PosL from, PosL to) {
    const int i = blockIdx.x * kAtomThreads + threadIdx.x;
    if (i >= ntp)
        return;
    double a, b, c;
    from.get(i, a, b, c);
    to.put(i, a, b, c);
}

// The NaN sentinel atom at slot nt of a position buffer.
__global__ void k_put_sentinel(int nt, PosL p) {
    const double nan = __builtin_nan("");
    p.put(nt, nan, nan, nan);
}

// ------------------------------------------------------------------ binning

// Cell slot of every atom and its (arbitrary) arrival rank within the cell.
__global__ __launch_bounds__(kAtomThreads) void k_bin_count(Dims d, const Box *__restrict__ boxes,
                                                            const int32_t *__restrict__ atom_box, PosL P,
                                                            int32_t *cell_of, int32_t *slot, int32_t *cell_count,
                                                            int32_t *err) {
    const int i = blockIdx.x * kAtomThreads + threadIdx.x;
    if (i >= d.nt)
        return;
    const Box &B = boxes[atom_box[i]];
    // positions drift unwrapped between list builds
    double px, py, pz;
    P.get(i, px, py, pz);
    px = wrap(px, B.L);
    py = wrap(py, B.L);
    pz = wrap(pz, B.L);
    if (!(isfinite(px) && isfinite(py) && isfinite(pz)))
        atomicOr(err, kErrNonFinite);
    const int sx = sub_coord(px, B.hside, B.nc), sy = sub_coord(py, B.hside, B.nc),
              sz = sub_coord(pz, B.hside, B.nc);
    const int c = cell_slot(B, sx >> 1, sy >> 1, sz >> 1) * kSub + ((sz & 1) * 2 + (sy & 1)) * 2 + (sx & 1);
    cell_of[i] = c;  // bin slot: cell slot and subcell
    // One atomic per distinct bin of the wavefront (atoms arrive nearly
    // bin-sorted, so a wavefront spans a few dozen subcells): a first pass
    // over the wave's distinct bins (no memory traffic) gives each lane its
    // bin's leader, lane count and its rank among them; then every leader
    // issues its atomic at once, so the wavefront waits for one round trip
    // instead of one per bin, and each lane takes slot base + rank.  (The
    // slot order within a bin is arbitrary; the later rank by original id
    // makes it deterministic.)
    const int lane = threadIdx.x & 63;
    uint64_t todo = __ballot(1);
    int rank = 0, cnt = 0, leader = lane;
    while (todo) {
        const int first = __builtin_ctzll(todo);
        const int c0 = __shfl(c, first, 64);
        const uint64_t m = __ballot(c == c0);
        if (c == c0) {
            leader = first;
            cnt = __popcll(m);
            rank = __popcll(m & ((uint64_t(1) << lane) - 1));
        }
        todo &= ~m;
    }
    int base = 0;
    if (lane == leader)
        base = atomicAdd(&cell_count[c], cnt);
    slot[i] = __shfl(base, leader, 64) + rank;
}

// Exclusive scan, pass 1: each workgroup scans a tile of kScanTile counts
// (four per thread), records the tile total and clears the counts for the
// next binning (so that binning needs no separate fill).
__global__ __launch_bounds__(256) void k_scan_tiles(int32_t *__restrict__ in, int32_t *__restrict__ out,
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
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (base + q < n)
            in[base + q] = 0;
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

// The whole scan in one workgroup, for up to kScanOne counts: each thread
// sums a contiguous run of at most kScanOne / 1024 of them, the workgroup
// scans the run totals, and each thread reads its run again (from the
// cache), writes its offsets to cell_start[0..n] and clears its counts for
// the next binning (so that binning needs no separate fill).  The run is
// read in batches of 32 whose loads are all in flight together.  Each
// thread's run is contiguous, so a wavefront's loads and stores touch one
// cache line per lane: beyond a few tens of thousands of counts the
// coalesced multi-workgroup scan is faster (measured: 64k counts took
// 150 us here).
__global__ __launch_bounds__(1024) void k_scan_one(int32_t *counts, int32_t *out, int n) {
    constexpr int M = 32;
    __shared__ int32_t sh[32];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;  // <= kScanOne / 1024
    const int b0 = t * per, b1 = min(b0 + per, n);
    int tot = 0;
    for (int base = b0; base < b1; base += M) {
        int v[M];
#pragma unroll
        for (int q = 0; q < M; ++q)
            v[q] = base + q < b1 ? counts[base + q] : 0;
#pragma unroll
        for (int q = 0; q < M; ++q)
            tot += v[q];
    }
    // run totals scanned within each wavefront, then across the 16 of them
    const int lane = t & 63, wv = t >> 6;
    const int incl = wave_prefix_incl(tot);
    if (lane == 63)
        sh[wv] = incl;
    __syncthreads();
    if (wv == 0) {
        const int w = lane < 16 ? sh[lane] : 0;
        const int wi = wave_prefix_incl(w);
        if (lane < 16)
            sh[16 + lane] = wi - w;
    }
    __syncthreads();
    int run = sh[16 + wv] + incl - tot;
    for (int base = b0; base < b1; base += M) {
        int v[M];
#pragma unroll
        for (int q = 0; q < M; ++q)
            v[q] = base + q < b1 ? counts[base + q] : 0;
#pragma unroll
        for (int q = 0; q < M; ++q)
            if (base + q < b1) {
                out[base + q] = run;
                counts[base + q] = 0;
                run += v[q];
            }
    }
    if (t == 1023)
        out[n] = run;
}

// Pass 2: each workgroup (256 counts, inside one tile) sums the totals of
// the tiles before its own and adds that to its offsets; workgroup 0 also
// writes the grand total to out[n].
__global__ __launch_bounds__(256) void k_scan_add(int32_t *out, const int32_t *__restrict__ sums, int ntile,
                                                  int n) {
    __shared__ int32_t sh[2][4];
    const int t = threadIdx.x, tile = blockIdx.x * 256 / kScanTile;
    int before = 0, all = 0;
    for (int k = t; k < ntile; k += 256) {
        const int v = sums[k];
        before += k < tile ? v : 0;
        all += v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        before += __shfl_xor(before, o, 64);
        all += __shfl_xor(all, o, 64);
    }
    if ((t & 63) == 0) {
        sh[0][t >> 6] = before;
        sh[1][t >> 6] = all;
    }
    __syncthreads();
    before = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    const int i = blockIdx.x * 256 + t;
    if (i < n)
        out[i] += before;
    if (blockIdx.x == 0 && t == 0)
        out[n] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
}

__global__ __launch_bounds__(kAtomThreads) void k_scatter(int n, const int32_t *__restrict__ cell_of,
                                                          const int32_t *__restrict__ slot,
                                                          const int32_t *__restrict__ cell_start, int32_t *tmp_idx) {
    const int i = blockIdx.x * kAtomThreads + threadIdx.x;
    if (i < n)
        tmp_idx[cell_start[cell_of[i]] + slot[i]] = i;
}

// Atomic arrival order inside a bin (a cell's subcell) is not reproducible:
// each atom's final place is its bin start plus the number of bin members
// with a smaller original id.  Then positions, velocities and ids move to that place.  The
// ids of the workgroup's own arrival slots are staged in LDS first, so only
// cells that straddle a workgroup boundary read members from global memory.
__global__ __launch_bounds__(kAtomThreads) void k_rank_permute(
    int n, int nbox, const Box *__restrict__ boxes, const int32_t *__restrict__ atom_box, const int32_t *__restrict__ tmp_idx,
    const int32_t *__restrict__ cell_of,
    const int32_t *__restrict__ cell_start, PosL P, const double *__restrict__ vx, const double *__restrict__ vy,
    const double *__restrict__ vz, const int32_t *__restrict__ orig, PosL P2, double *vx2, double *vy2,
    double *vz2, int32_t *orig2) {
    __shared__ int32_t keys[kAtomThreads];
    const int q0 = blockIdx.x * kAtomThreads, q = q0 + threadIdx.x;
    const int p = q < n ? tmp_idx[q] : 0;
    const int key = q < n ? orig[p] : 0;
    keys[threadIdx.x] = key;
    __syncthreads();
    if (q >= n)
        return;
    // everything that depends only on the source slot is requested at once
    const int c = cell_of[p];
    const double L = boxes[nbox == 1 ? 0 : atom_box[p]].L;  // a box keeps its slot range
    double px, py, pz;
    P.get(p, px, py, pz);
    const double pvx = vx[p], pvy = vy[p], pvz = vz[p];
    const int b = cell_start[c], e = cell_start[c + 1];
    int rank = 0;
    for (int r = b; r < e; ++r) {
        const int kr = (r >= q0 && r < q0 + kAtomThreads) ? keys[r - q0] : orig[tmp_idx[r]];
        rank += int(kr < key);
    }
    const int dst = b + rank;
    P2.put(dst, wrap(px, L), wrap(py, L), wrap(pz, L));
    vx2[dst] = pvx;
    vy2[dst] = pvy;
    vz2[dst] = pvz;
    orig2[dst] = key;
}

// ------------------------------------------------------------------ neighbor list

// Descriptor of the box that block b belongs to (a single box needs no
// lookup, which saves a dependent memory round trip at every workgroup start).
__device__ __forceinline__ Box block_box(const Dims &d, const Box *__restrict__ boxes,
                                         const int32_t *__restrict__ blk_box, int b) {
    return boxes[d.nbox == 1 ? 0 : blk_box[b]];
}

// Neighbor-list build.  Every j != i within (cutoff + skin) of i enters i's
// list (Sec. 3.2, Fig. 1).  The cells are cut in 2 x 2 x 2 subcells of side
// >= (cutoff + skin) / 2 - smaller cells with a larger stencil, as the
// footnote to Fig. 1 allows - so every partner lies within +-2 subcells
// along each axis: 125 subcells, about 0.56 of the volume of the 27 cells
// (boxes of two cells per axis have four distinct subcells per axis, all
// of them).  Candidates are visited in one canonical order, the same on
// every path and schedule: for dz, then dy, then dx in -2 .. 2 (distinct
// subcells only, in that order), the subcell's atoms in memory order (bins
// are sorted by original id).  So lists, and the force sums that follow
// them, do not depend on the schedule.
//
// Subcell rows (the common path): the workgroup copies its neighborhood
// into LDS ordered by subcell rows (z, then y, then x fastest), so the x
// subcells of each of i's (y, z) rows are one run of consecutive slots (two
// where a small box's row wraps).  Each lane walks its own runs back to
// back, four candidates per round, so short runs cost no wait for the
// wavefront's longest run.  Next to each position the copy keeps the
// atom's slot in the force kernel's neighborhood copy (cells in table
// order), which is what the list stores.
//
// Global gathers: neighborhoods too crowded for the row copy (26 bytes a
// slot and the subcell offsets, within the area sized for the force
// kernel's 24) read candidates from memory in the same order; they store
// force-kernel slots when the force kernel stages the neighborhood, else
// 32-bit global indices.
typedef __attribute__((address_space(3))) uint16_t lds_u16;

// Exclusive prefix sum of n 16-bit counts in LDS, in place, with a[n] = the
// total; wsum is LDS scratch of kMaxThreads / 64 ints.  Ends with a barrier.
__device__ __forceinline__ void scan_excl_u16(lds_u16 *a, int n, int *wsum) {
    const int T = blockDim.x, K = (n + T - 1) / T, b0 = threadIdx.x * K;
    int tot = 0;
    for (int q = 0; q < K; ++q)
        tot += (b0 + q < n) ? int(a[b0 + q]) : 0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int incl = wave_prefix_incl(tot);
    if (lane == 63)
        wsum[wv] = incl;
    __syncthreads();
    int run = incl - tot;
    for (int w = 0; w < wv; ++w)
        run += wsum[w];
    for (int q = 0; q < K; ++q)
        if (b0 + q < n) {
            const int v = a[b0 + q];
            a[b0 + q] = uint16_t(run);
            run += v;
        }
    if (threadIdx.x == T - 1)
        a[n] = uint16_t(run);
    __syncthreads();
}

// Subcell grid of a block neighborhood.  Along each axis the neighborhood
// holds the distinct cells c0 - 1, c0, ... (periodic), n = min(e + 2, nc)
// of them (hood_axes() lists them in this order), two subcells each: grid
// index g along an axis is the box subcell (2 c0 - 2 + g) mod 2 nc.
struct SubGrid {
    int c0[3];  // first own cell per axis
    int n[3];   // neighborhood cells per axis
    int nx, ny, nz, ng;
    int nsub;   // subcells per box axis, 2 nc
    int m;      // distinct stencil subcells per axis: min(5, nsub)
};

__device__ __forceinline__ SubGrid sub_grid(const Box &B, int lb) {
    SubGrid G;
    const int nbx = B.nbx;
    const int bc[3] = {lb % nbx, (lb / nbx) % nbx, lb / (nbx * nbx)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        G.c0[a] = B.edge * bc[a];
        G.n[a] = min(min(B.edge, B.nc - G.c0[a]) + 2, B.nc);
    }
    G.nx = 2 * G.n[0];
    G.ny = 2 * G.n[1];
    G.nz = 2 * G.n[2];
    G.ng = G.nx * G.ny * G.nz;
    G.nsub = 2 * B.nc;
    G.m = min(5, G.nsub);
    return G;
}

__device__ __forceinline__ int wrap_index(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Bin slot of grid subcell g, and the neighborhood cell (table index) it
// lies in.
__device__ __forceinline__ int sub_bin(const Box &B, const SubGrid &G, int g, int &u) {
    const int gx = g % G.nx, r = g / G.nx, gy = r % G.ny, gz = r / G.ny;
    const int kx = gx >> 1, ky = gy >> 1, kz = gz >> 1;
    const int cx = wrap_index(G.c0[0] - 1 + kx, B.nc), cy = wrap_index(G.c0[1] - 1 + ky, B.nc),
              cz = wrap_index(G.c0[2] - 1 + kz, B.nc);
    u = (kz * G.n[1] + ky) * G.n[0] + kx;
    return cell_slot(B, cx, cy, cz) * kSub + ((gz & 1) * 2 + (gy & 1)) * 2 + (gx & 1);
}

// Copy the neighborhood into LDS in subcell-row order: positions at S (24
// bytes a slot) and each atom's slot in the force kernel's copy at F;
// soff[g] = first slot of grid subcell g, soff[ng] = atoms staged.  Ends
// with a barrier.
__device__ __forceinline__ void sub_stage(const Box &B, const SubGrid &G, const Hood &h,
                                          const int32_t *__restrict__ cell_start, const PosL &P, lds_double *S,
                                          lds_u16 *F, lds_u16 *soff, int *wsum) {
    const int T = blockDim.x;
    for (int g = threadIdx.x; g < G.ng; g += T) {
        int u;
        const int bs = sub_bin(B, G, g, u);
        soff[g] = uint16_t(cell_start[bs + 1] - cell_start[bs]);
    }
    __syncthreads();
    scan_excl_u16(soff, G.ng, wsum);
    for (int g = threadIdx.x; g < G.ng; g += T) {
        int u;
        const int bs = sub_bin(B, G, g, u);
        const int st = cell_start[bs], n = cell_start[bs + 1] - st;
        const int dst = soff[g], fb = h.off[u] + (st - h.cs[u]);
        for (int k = 0; k < n; ++k) {
            lds_double *a = lds_slot(S, dst + k);
            double px, py, pz;
            P.get(st + k, px, py, pz);
            a[0] = px;
            a[1] = py;
            a[2] = pz;
            F[dst + k] = uint16_t(fb + k);
        }
    }
    __syncthreads();
}

// Distance test of a candidate: MIC takes the minimum image of the raw
// difference; without it no raw difference along an axis exceeds L/2.
template <bool MIC>
__device__ __forceinline__ double cand_dist2(double xi, double yi, double zi, double xj, double yj, double zj,
                                             const Box &B) {
    double dx, dy, dz;
    if (MIC)
        return pair_delta(xi, yi, zi, xj, yj, zj, B.L, B.halfL, B.halfL2, dx, dy, dz);
    return dist2(xi - xj, yi - yj, zi - zj);
}

// Element of entry k of a 16-bit list relative to the atom's entry 0
// (nbr_index16(i, k, n) - nbr_index16(i, 0, n): rows of eight entries, 64
// atoms to a row of the tile), in 32-bit unsigned arithmetic.
__device__ __forceinline__ unsigned entry16(int k) { return __umul24(unsigned(k) >> 3, 504u) + unsigned(k); }

// Entry c of the 16-bit list of the atom whose entry 0 is at wp, if it is
// within capacity.
__device__ __forceinline__ void put16(uint16_t *wp, int &c, int maxnb, int v) {
    if (c < maxnb)
        wp[entry16(c)] = uint16_t(v);
    ++c;
}

// Where atom i's runs lie in the subcell-row copy: grid coordinates of the
// current row, the first subcell of its x-run, the stencil offsets walked so
// far, and the run's split where a small box's row wraps.
struct RowWalk {
    int gz, gy, xs;  // grid z, y of the current row; grid x of the run's first subcell
    int kz, ky;      // stencil offsets walked so far along z, y
    int xa, xb;      // run lengths in subcells: [xs, xs + xa), then [0, xb) where the row wraps
    int piece;       // 0: first part of the row, 1: the wrapped part
};

// Slots [t, e) of the run w points at.
__device__ __forceinline__ void row_run(const SubGrid &G, const lds_u16 *soff, const RowWalk &w, int &t, int &e) {
    const int rb = (w.gz * G.ny + w.gy) * G.nx;
    const int a = rb + (w.piece ? 0 : w.xs), len = w.piece ? w.xb : w.xa;
    t = soff[a];
    e = soff[a + len];
}

// The run after w's (selects only); false after the last.
__device__ __forceinline__ bool row_next(const SubGrid &G, int gy0, RowWalk &w) {
    const bool second = w.piece == 0 && w.xb > 0;  // the wrapped part of this row
    const bool newz = !second && w.ky + 1 == G.m;
    const bool last = newz && w.kz + 1 == G.m;
    const int gy1 = w.gy + 1 == G.ny ? 0 : w.gy + 1, gz1 = w.gz + 1 == G.nz ? 0 : w.gz + 1;
    w.gy = second ? w.gy : (newz ? gy0 : gy1);
    w.ky = second ? w.ky : (newz ? 0 : w.ky + 1);
    w.gz = newz && !last ? gz1 : w.gz;
    w.kz = newz && !last ? w.kz + 1 : w.kz;
    w.piece = second ? 1 : 0;
    return !last;
}

// Kinds of block for the list build's row walk.
enum { kRowsInterior = 0, kRowsFace = 1, kRowsWrap = 2 };

// Which of the 25 rows of atom i's 5 x 5 x 5 subcell stencil its cutoff
// sphere reaches, and how far along x in each.  Along one axis the atom lies
// at distance q from the low edge of its own subcell (side hs); the
// subcells at offsets -2, -1, +1, +2 begin q + hs, q, hs - q and 2 hs - q
// away.  A row (offsets dy, dz) is needed if its nearest point lies within
// the cutoff, and in a needed row the x-run keeps the subcells at offsets
// -2 and -1 (+1 and +2) while theirs do: the needed subcells of a row are
// contiguous around dx = 0.  Every atom in a subcell left out is farther than
// rl from i by more than the rounding of its difference (the test admits
// rounding through a margin far above it), so the distance test would reject
// it: leaving it out changes no list.  Bit r of need marks row r = 5 kz + ky;
// four bits per row in lo and hi (two for the offsets kept below x = 0, two
// above).
struct RowTrim {
    unsigned need;
    uint64_t lo, hi;  // codes of rows 0-15 and 16-24 (no indexed array: it would live in scratch memory)
};

__device__ __forceinline__ RowTrim row_trim(double xi, double yi, double zi, int X, int Y, int Z, const Box &B) {
    const double hs = B.hside;
    // rounding of positions and subcell edges stays below a few ulp(L)
    const double R = B.rl2 + 2e-12 * B.L * sqrt(B.rl2);
    auto q5 = [&](double p, int s, double q[5]) {
        const double o = p - double(s) * hs;
        const double lo1 = max(o, 0.0), hi1 = max(hs - o, 0.0);
        q[0] = (lo1 + hs) * (lo1 + hs);
        q[1] = lo1 * lo1;
        q[2] = 0.0;
        q[3] = hi1 * hi1;
        q[4] = (hi1 + hs) * (hi1 + hs);
    };
    double qx[5], qy[5], qz[5];
    q5(xi, X, qx);
    q5(yi, Y, qy);
    q5(zi, Z, qz);
    RowTrim T;
    T.need = 0;
    T.lo = T.hi = 0;
#pragma unroll
    for (int kz = 0; kz < 5; ++kz)
#pragma unroll
        for (int ky = 0; ky < 5; ++ky) {
            const int r = 5 * kz + ky;
            const double dyz = qy[ky] + qz[kz];
            const unsigned lo = (qx[0] + dyz < R) ? 2u : ((qx[1] + dyz < R) ? 1u : 0u);
            const unsigned hi = (qx[4] + dyz < R) ? 2u : ((qx[3] + dyz < R) ? 1u : 0u);
            T.need |= (dyz < R ? 1u : 0u) << r;
            const uint64_t cr = uint64_t(lo | (hi << 2));
            if (r < 16)
                T.lo |= cr << (4 * r);
            else
                T.hi |= cr << (4 * (r - 16));
        }
    return T;
}

// Atom i's runs in the subcell-row copy, one lane per atom (BL = 1) or two
// lanes testing alternate candidates (BL = 2, lane p).  A round reads four
// (eight) consecutive slots unconditionally, up to three (seven) past the
// run's end, which the t < e test rejects; the self test compares the
// force-kernel slot.  Every round also looks up where the next run lies and
// takes it if this one is done: one straight loop, so a lane whose run
// ended moves on while the others finish theirs (branching to the next run
// instead lets the compiler nest a loop over each run's rounds, which the
// whole wavefront then waits out).
//
// GEOM says how the differences get their periodic images:
//   kRowsInterior: the neighborhood crosses no face of the box, so no raw
//     difference exceeds L/2;
//   kRowsFace: the neighborhood crosses a face but holds no cell twice.  A
//     candidate's image is then fixed by where its subcell sits in the grid:
//     subcells before grid index bl (past the low face) take d - (-L),
//     subcells from bh on (past the high face) take d - L, the rest d - 0.
//     For every candidate this is the oracle's shift (d > L/2: d -= L; d <
//     -L/2: d += L), applied to the same raw difference, so decisions and
//     roundings are the oracle's: along y and z the shift is the row's,
//     along x it changes at most once inside a run, at slot tw;
//   kRowsWrap: the neighborhood holds every cell of some axis (small
//     boxes): rows and runs wrap, and each difference takes the minimum
//     image of its value.
// The first two walk the rows and x-runs of row_trim(); the third the
// whole stencil.  HALF (first two only): a candidate in one of the block's
// own cells is kept only if its force-kernel slot exceeds i's, and its
// entry carries bit 15 (the partner takes the reaction); along a row the
// own cells' slots are [to0, to1).  Returns the number of neighbors found.
template <int BL, int GEOM, bool HALF = false>
__device__ __forceinline__ int build_rows(lds_double *S, const lds_u16 *F, const lds_u16 *soff, const SubGrid &G,
                                          int gx, int gy, int gz, int fself, double xi, double yi, double zi,
                                          const RowTrim &T, const Box &B, int maxnb, int p, uint16_t *nbr16, int i,
                                          int nchunk) {
    constexpr bool WRAP = GEOM == kRowsWrap, SHIFT = GEOM == kRowsFace;
    RowWalk w;
    w.gz = wrap_index(gz - 2, G.nz);
    w.gy = wrap_index(gy - 2, G.ny);
    w.xs = wrap_index(gx - 2, G.nx);
    w.xa = min(G.m, G.nx - w.xs);
    w.xb = G.m - w.xa;
    w.kz = w.ky = w.piece = 0;
    const int gy0 = w.gy;
    // without wrapping: row r = 5 kz + ky of the stencil starts at table
    // index base + kz nx ny + ky nx (its subcell at x offset -2)
    const int base = ((gz - 2) * G.ny + (gy - 2)) * G.nx + (gx - 2), zstride = G.nx * G.ny;
    // face shifts: grid indices below bl lie past the low face, from bh on
    // past the high face (per axis)
    const int blx = 2 - 2 * G.c0[0], bhx = G.nsub - 2 * G.c0[0] + 2;
    const int bly = 2 - 2 * G.c0[1], bhy = G.nsub - 2 * G.c0[1] + 2;
    const int blz = 2 - 2 * G.c0[2], bhz = G.nsub - 2 * G.c0[2] + 2;
    // along x: slots before tw take sxa, the others sxb; tw sits at grid
    // index gx - 2 + dgb of each row
    double sxa = 0.0, sxb = 0.0;
    int dgb = 0, tw = -1;
    if (SHIFT) {
        if (blx > gx - 2) {
            sxa = -B.L;
            dgb = blx - (gx - 2);
        } else if (bhx <= gx + 2) {
            sxb = B.L;
            dgb = bhx - (gx - 2);
        }
    }
    const bool xshift = SHIFT && (sxa != 0.0 || sxb != 0.0);
    auto shift_of = [&](int g, int bl, int bh) { return g < bl ? -B.L : (g >= bh ? B.L : 0.0); };
    double sy = 0.0, sz = 0.0;
    int to0 = 0, to1 = 0;
    // slots [t, e) of stencil row r, tw for it and its own slots [to0, to1)
    auto trim_run = [&](int r, int &t_, int &e_, int &tw_, double &sy_, double &sz_, int &to0_, int &to1_) {
        const int kz = (r * 13) >> 6, ky = r - 5 * kz;  // r / 5, r % 5 for r < 25
        const unsigned c = unsigned((r < 16 ? T.lo : T.hi) >> ((r & 15) * 4)) & 15u;
        const int rb = base + kz * zstride + ky * G.nx;
        t_ = soff[rb + 2 - int(c & 3u)];
        e_ = soff[rb + 3 + int(c >> 2)];
        if (SHIFT) {
            tw_ = xshift ? int(soff[rb + dgb]) : -1;
            sy_ = shift_of(gy - 2 + ky, bly, bhy);
            sz_ = shift_of(gz - 2 + kz, blz, bhz);
        }
        if (HALF) {
            // own cells: neighborhood coordinates 1..n - 2, grid subcells
            // 2..2n - 3 per axis
            const int cy = (gy - 2 + ky) >> 1, cz = (gz - 2 + kz) >> 1;
            const bool rown = cy >= 1 && cy <= G.n[1] - 2 && cz >= 1 && cz <= G.n[2] - 2;
            const int r0 = rb - (gx - 2);  // the row's grid x = 0
            const int a0 = soff[r0 + 2], a1 = soff[r0 + 2 * G.n[0] - 2];
            to0_ = rown ? a0 : 0;
            to1_ = rown ? a1 : 0;
        }
    };
    int t, e, row = 0;
    if (WRAP) {
        row_run(G, soff, w, t, e);
    } else {
        row = __builtin_ctz(T.need);  // the centre row is always needed
        trim_run(row, t, e, tw, sy, sz, to0, to1);
    }
    // whether slot tt is kept, and its list entry
    auto keep = [&](int tt, int fj, bool near, uint16_t &v) {
        if (HALF) {
            const bool own = tt >= to0 && tt < to1;
            v = uint16_t(fj | (own ? 0x8000 : 0));
            return near && (own ? fj > fself : fj != fself);
        }
        v = uint16_t(fj);
        return near && fj != fself;
    };
    // difference of one candidate along the three axes, with its image
    auto dist = [&](double xj, double yj, double zj, int tj) {
        if (WRAP)
            return cand_dist2<true>(xi, yi, zi, xj, yj, zj, B);
        if (SHIFT) {
            const double dx = (xi - xj) - (tj < tw ? sxa : sxb);
            const double dy = (yi - yj) - sy;
            const double dz = (zi - zj) - sz;
            return dist2(dx, dy, dz);
        }
        return dist2(xi - xj, yi - yj, zi - zj);
    };
    int c = 0;
    uint16_t *const wp = nbr16 + nbr_index16(i, 0, nchunk);
    for (;;) {
        // the round's candidates: slots t .. t + 3 (BL = 1), or the lane's
        // four of slots t .. t + 7 (BL = 2)
        double px[4], py[4], pz[4];
        int tr[4];
        {
            const int t0 = BL == 1 ? t : t + p;
            const lds_char *pb = (const lds_char *)S + __umul24(unsigned(t0), 24u);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const lds_double *q = (const lds_double *)(pb + r * 24 * BL);
                px[r] = q[0];
                py[r] = q[1];
                pz[r] = q[2];
                tr[r] = F[t0 + BL * r];
            }
        }
        // where the run after this one lies (taken below once this one is
        // done), looked up ahead of the round's tests so that its LDS reads
        // overlap them instead of ending the round
        int nt, ne;
        bool more;
        RowWalk w2 = w;
        int nrow = row, ntw = tw, nto0 = to0, nto1 = to1;
        double nsy = sy, nsz = sz;
        if (WRAP) {
            more = row_next(G, gy0, w2);
            row_run(G, soff, w2, nt, ne);
        } else {
            // the next needed row (row itself when there is none)
            const unsigned rest = row < 24 ? T.need & (~0u << (row + 1)) : 0u;
            more = rest != 0u;
            nrow = more ? __builtin_ctz(rest) : row;
            trim_run(nrow, nt, ne, ntw, nsy, nsz, nto0, nto1);
        }
        if (BL == 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double s = dist(px[r], py[r], pz[r], t + r);
                uint16_t v;
                if (keep(t + r, tr[r], s < B.rl2 && t + r < e, v))
                    put16(wp, c, maxnb, v);
            }
            t += 4;
        } else {
            unsigned mine = 0;  // bit 2r + p: slot t + 2r + p accepted
            uint16_t vr[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double s = dist(px[r], py[r], pz[r], t + 2 * r + p);
                mine |= keep(t + 2 * r + p, tr[r], s < B.rl2 && t + 2 * r + p < e, vr[r]) ? (1u << (2 * r + p)) : 0u;
            }
            const unsigned m8 = mine | unsigned(__shfl_xor(int(mine), 1, 64));
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 2 * r + p;
                if (mine & (1u << j)) {
                    const int pos = c + __popc(m8 & ((1u << j) - 1u));
                    if (pos < maxnb)
                        wp[entry16(pos)] = vr[r];
                }
            }
            c += __popc(m8);
            t += 8;
        }
        const bool adv = t >= e;
        if (WRAP) {
            w.gz = adv ? w2.gz : w.gz;
            w.gy = adv ? w2.gy : w.gy;
            w.kz = adv ? w2.kz : w.kz;
            w.ky = adv ? w2.ky : w.ky;
            w.piece = adv ? w2.piece : w.piece;
        } else {
            if (SHIFT) {
                sy = adv ? nsy : sy;
                sz = adv ? nsz : sz;
                tw = adv ? ntw : tw;
            }
            if (HALF) {
                to0 = adv ? nto0 : to0;
                to1 = adv ? nto1 : to1;
            }
            row = adv ? nrow : row;
        }
        if (adv && !more)
            break;
        t = adv ? nt : t;
        e = adv ? ne : e;
    }
    return c;
}

// Atom i's candidates from memory, in the canonical order (the atom's
// first lane alone).  fits: store force-kernel slots (16-bit), else global
// indices (32-bit).  Returns the number of neighbors found.
__device__ __forceinline__ int build_global(const Box &B, const SubGrid &G, const Hood &h, bool fits,
                                            const int32_t *__restrict__ cell_start, const PosL &P, int i,
                                            double xi, double yi, double zi, int X, int Y, int Z, int maxnb,
                                            int32_t *__restrict__ nbr, int nchunk) {
    uint16_t *nbr16 = reinterpret_cast<uint16_t *>(nbr);
    int c = 0;
    for (int kz = 0; kz < G.m; ++kz) {
        const int sz = wrap_index(Z - 2 + kz, G.nsub);
        for (int ky = 0; ky < G.m; ++ky) {
            const int sy = wrap_index(Y - 2 + ky, G.nsub);
            for (int kx = 0; kx < G.m; ++kx) {
                const int sx = wrap_index(X - 2 + kx, G.nsub);
                const int cx = sx >> 1, cy = sy >> 1, cz = sz >> 1;
                const int bs = cell_slot(B, cx, cy, cz) * kSub + ((sz & 1) * 2 + (sy & 1)) * 2 + (sx & 1);
                const int st = cell_start[bs], en = cell_start[bs + 1];
                // table index of the cell: its place along each neighborhood axis
                const int u = (wrap_index(cz - G.c0[2] + 1, B.nc) * G.n[1] + wrap_index(cy - G.c0[1] + 1, B.nc)) *
                                  G.n[0] +
                              wrap_index(cx - G.c0[0] + 1, B.nc);
                const int fb = h.off[u] - h.cs[u];
                for (int g = st; g < en; ++g) {
                    double dx, dy, dz, xj, yj, zj;
                    P.get(g, xj, yj, zj);
                    const double s = pair_delta(xi, yi, zi, xj, yj, zj, B.L, B.halfL, B.halfL2, dx, dy, dz);
                    if (s < B.rl2 && g != i) {
                        if (c < maxnb) {
                            if (fits)
                                nbr16[nbr_index16(i, c, nchunk)] = uint16_t(fb + g);
                            else
                                nbr[nbr_index(i, c, nchunk)] = g;
                        }
                        ++c;
                    }
                }
            }
        }
    }
    return c;
}

template <int BL, int LAY>
__global__ __launch_bounds__(kMaxThreads) void k_build(Dims d, const Box *__restrict__ boxes,
                                                       const int32_t *__restrict__ blk_box,
                                                       const double *__restrict__ pin,
                                                       const int32_t *__restrict__ cell_start,
                                                       int32_t *__restrict__ hood_tab, int32_t *__restrict__ cnt,
                                                       int32_t *__restrict__ nbr, int32_t *err) {
    __shared__ Hood h;
    __shared__ int wsum[kMaxThreads / 64];
    extern __shared__ double lds[];
    int b, part;
    if (!block_part(d, b, part))
        return;
    const Box B = block_box(d, boxes, blk_box, b);
    const int lb = b - B.block_off;
    hood_setup(B, lb, cell_start, h);
    if (part == 0)
        hood_store(h, b, hood_tab);
    int lo, hi;
    h.share(part, d.parts, lo, hi);
    const int total = h.off[h.ncell];
    const bool fits = total <= d.cap;
    const SubGrid G = sub_grid(B, lb);
    // the row copy takes 26 bytes a slot (position, force-kernel slot) and
    // the subcell offsets, within the area sized for the force kernel
    const int nslot = total + 2 + kHoodPad;
    const bool rows = fits && 26 * nslot + 2 * (G.ng + 1) <= 24 * (d.cap + 2 + kHoodPad);
    lds_double *S = (lds_double *)lds;
    lds_u16 *F = (lds_u16 *)((lds_char *)lds + 24 * nslot);
    lds_u16 *soff = F + nslot;
    if (rows)
        sub_stage(B, G, h, cell_start, pos_of(LAY, d.ntp, pin), S, F, soff, wsum);
    // list padding points at the NaN sentinel: force-kernel LDS slot cap, or
    // global slot nt
    const int sentinel = fits ? d.cap : d.nt;
    uint16_t *nbr16 = reinterpret_cast<uint16_t *>(nbr);
    // interior: no neighborhood cell range crosses a face of the box.  A
    // candidate lies within two subcells of its atom's subcell, less than
    // 1.5 cells away along each axis, and a neighborhood that holds no cell
    // twice needs at least four cells per axis (L/2 >= 2 cells): no raw
    // difference exceeds L/2
    bool interior = true, wraps = false;
    for (int a = 0; a < 3; ++a) {
        const int c0 = G.c0[a], e = min(B.edge, B.nc - c0);
        interior &= c0 >= 1 && c0 + e <= B.nc - 1;
        wraps |= G.n[a] < e + 2;  // the neighborhood holds every cell of the axis
    }
    // half lists only on the row walk (the other paths list pairs in full,
    // which the force kernel handles alike)
    int s_lo, span;
    const bool half = rows && block_half(d, B, lb, h, fits, s_lo, span);
    const int p = threadIdx.x & (BL - 1);  // lane of the atom's pair (BL = 2)
    for (int i = lo + threadIdx.x / BL; i < hi; i += blockDim.x / BL) {
        double xi, yi, zi;
        pos_get(LAY, d.ntp, pin, i, xi, yi, zi);
        const int X = sub_coord(xi, B.hside, B.nc), Y = sub_coord(yi, B.hside, B.nc),
                  Z = sub_coord(zi, B.hside, B.nc);
        int c = 0;
        if (rows) {
            // grid subcell of i
            const int gx = wrap_index(X - 2 * G.c0[0] + 2, G.nx), gy = wrap_index(Y - 2 * G.c0[1] + 2, G.ny),
                      gz = wrap_index(Z - 2 * G.c0[2] + 2, G.nz);
            const int us = ((gz >> 1) * G.n[1] + (gy >> 1)) * G.n[0] + (gx >> 1);
            const int fself = h.off[us] + (i - h.cs[us]);
            RowTrim T{};
            if (!wraps)
                T = row_trim(xi, yi, zi, X, Y, Z, B);
#define TMD_ROWS(GEOM, HALF)                                                                                        \
    build_rows<BL, GEOM, HALF>(S, F, soff, G, gx, gy, gz, fself, xi, yi, zi, T, B, d.maxnb, p, nbr16, i, d.nchunk)
            if (wraps)
                c = TMD_ROWS(kRowsWrap, false);
            else if (interior)
                c = half ? TMD_ROWS(kRowsInterior, true) : TMD_ROWS(kRowsInterior, false);
            else
                c = half ? TMD_ROWS(kRowsFace, true) : TMD_ROWS(kRowsFace, false);
#undef TMD_ROWS
        } else if (p == 0) {
            c = build_global(B, G, h, fits, cell_start, pos_of(LAY, d.ntp, pin), i, xi, yi, zi, X, Y, Z, d.maxnb,
                             nbr, d.nchunk);
        }
        if (p != 0)
            continue;  // the pair's first lane holds the same count and finishes the list
        const int stored = c < d.maxnb ? c : d.maxnb;
        cnt[i] = stored;
        // pad the last chunk and one whole chunk after it (every list has
        // room for it: nchunk = ceil(maxnb / 4) + 1); force loops read that
        // chunk in place of any chunk past the end
        if (fits) {
            // (at least through row 7, or the whole area when it has fewer
            // rows: with up to four lanes per atom the force kernel loads
            // rows 0 to 7 before it knows the count)
            const int pad_end = min(max(((stored + 7) & ~7) + 8, 64), 8 * d.nchunk);
            for (int k = stored; k < pad_end; ++k)
                nbr16[nbr_index16(i, k, d.nchunk)] = uint16_t(sentinel);
        } else {
            for (int k = stored; k < ((stored + 3) & ~3) + 4; ++k)
                nbr[nbr_index(i, k, d.nchunk)] = sentinel;
        }
        if (c > d.maxnb) {
            atomicOr(err, kErrOverflow);
            atomicMax(err + 1, c);
        }
    }
}

// ------------------------------------------------------------------ force

typedef int v4i __attribute__((ext_vector_type(4)));

// Positions of two list entries.
struct Duo {
    double x[2], y[2], z[2];
};

template <class POS>
__device__ __forceinline__ void fetch2(const POS &pos, int j0, int j1, Duo &q) {
    pos.get(j0, q.x[0], q.y[0], q.z[0]);
    pos.get(j1, q.x[1], q.y[1], q.z[1]);
}

// Two pairs of the sum F_i = sum f(s) d_ij over s < cutoff^2, with
// f = 48 eps sr6 (sr6 - 1/2) sr2 written as sr2 q (f12 q - f6), q = sr2^3,
// f12 = 48 eps sigma^12, f6 = 24 eps sigma^6 (Sec. 3.2, Eq. 2).  |d|^2 may
// use fused multiply-adds here: it decides only the cutoff test, whose pairs
// at s within an ulp of cutoff^2 have a vanishing share (the neighbor sets
// themselves come from the build's unfused sum).  mf6 and mu6 are -f6 and
// -u6.  A NaN sentinel entry fails both tests and adds nothing.  IMG: how
// the difference gets its periodic image (pair_geom: per pair, or from a
// neighborhood copy moved to its images near the block).
// HALF: the entries come from a half list (word: the two 16-bit entries,
// bit 15 marking a pair inside the block that the partner's list does not
// hold): such a pair also adds the reaction -f d to the partner's sum in R
// (LDS, index slot - s_lo), and its energy and virial count twice.
template <bool THERMO, int IMG, bool HALF = false>
__device__ __forceinline__ void eval2(const Duo &q, double xi, double yi, double zi, const Box &B, double mf6,
                                      double mu6, double &ax, double &ay, double &az, double &u, double &w,
                                      unsigned word = 0u, lds_double *R = nullptr, int s_lo = 0) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        double dx, dy, dz;
        const double s = pair_geom<IMG>(xi, yi, zi, q.x[m], q.y[m], q.z[m], B, dx, dy, dz);
        if (s < B.rc2) {
            const double sr2 = recip(s);
            const double q3 = sr2 * sr2 * sr2;
            const double f = (sr2 * q3) * fma(B.f12, q3, mf6);
            ax = fma(f, dx, ax);
            ay = fma(f, dy, ay);
            az = fma(f, dz, az);
            if (HALF) {
                const unsigned v = m ? word >> 16 : word & 0xFFFFu;
                const bool pair = (v & 0x8000u) != 0u;
                if (pair) {
                    lds_double *r = R + 3 * (int(v & 0x7FFFu) - s_lo);
                    __hip_atomic_fetch_add((double *)r, -f * dx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_add((double *)(r + 1), -f * dy, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_add((double *)(r + 2), -f * dz, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                if (THERMO) {
                    const double k = pair ? 2.0 : 1.0;
                    u = fma(k * q3, fma(B.u12, q3, mu6), u);
                    w = fma(k * s, f, w);
                }
            } else if (THERMO) {
                u = fma(q3, fma(B.u12, q3, mu6), u);
                w = fma(s, f, w);
            }
        }
    }
}

// Sum over one atom's list of 32-bit global indices (c entries in chunks of
// four), for blocks whose neighborhood does not fit in LDS: positions come
// from global memory.  With L lanes per atom the list is dealt in groups of
// eight entries (two chunks), lane p taking groups p, p + L, ... in order -
// the split and order of the 16-bit list's eight-entry chunks, so both give
// the same sums.  Every group below ceil(c / 8) is whole: the build pads a
// 32-bit list with NaN sentinel entries (global slot nt) through the chunk
// after its last one, and a sentinel adds nothing.  A plain loop: this path
// is rare, and a deeper pipeline here would set the register budget of the
// whole kernel.
template <bool THERMO>
__device__ __forceinline__ void pair_sum(const v4i *__restrict__ chunks, int p, int L, int c, const GlobalPos &pos,
                                         double xi, double yi, double zi, const Box &B, double mf6, double mu6,
                                         double &ax, double &ay, double &az, double &u, double &w) {
    const int ng = (c + 7) >> 3;
    for (int g = p; g < ng; g += L) {
        const v4i e0 = __builtin_nontemporal_load(chunks + (2 * g) * 64);
        const v4i e1 = __builtin_nontemporal_load(chunks + (2 * g + 1) * 64);
        Duo q;
        fetch2(pos, e0[0], e0[1], q);
        eval2<THERMO, 0>(q, xi, yi, zi, B, mf6, mu6, ax, ay, az, u, w);
        fetch2(pos, e0[2], e0[3], q);
        eval2<THERMO, 0>(q, xi, yi, zi, B, mf6, mu6, ax, ay, az, u, w);
        fetch2(pos, e1[0], e1[1], q);
        eval2<THERMO, 0>(q, xi, yi, zi, B, mf6, mu6, ax, ay, az, u, w);
        fetch2(pos, e1[2], e1[3], q);
        eval2<THERMO, 0>(q, xi, yi, zi, B, mf6, mu6, ax, ay, az, u, w);
    }
}

// Two LDS-slot entries packed in one 32-bit word of a 16-bit list, read
// from a neighborhood copy at LDS address 0 (the force kernel's layout):
// each slot's address, slot * 24, is one SDWA multiply that selects its half
// of the word, so a pair costs one address instruction (an added base would
// cost a second: the compiler does not fold the copy's base address into
// the reads' offset fields).  The three coordinates are three 8-byte reads:
// merged into a 16-byte read (x, y) plus z, two lanes whose slots differ by
// 11 or 21 modulo 32 collide in the LDS banks, and neighbors of adjacent
// atoms often sit that close; volatile keeps the compiler from merging them.
__device__ __forceinline__ void fetch2w(int word, Duo &q) {
    unsigned o0, o1;
    asm("v_mul_u32_u24_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_0 src1_sel:DWORD"
        : "=v"(o0)
        : "v"(word), "v"(24));
    asm("v_mul_u32_u24_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:DWORD"
        : "=v"(o1)
        : "v"(word), "v"(24));
    const volatile lds_double *a = reinterpret_cast<const volatile lds_double *>(uintptr_t(o0));
    const volatile lds_double *b = reinterpret_cast<const volatile lds_double *>(uintptr_t(o1));
    q.x[0] = a[0];
    q.y[0] = a[1];
    q.z[0] = a[2];
    q.x[1] = b[0];
    q.y[1] = b[1];
    q.z[1] = b[2];
}

// pair_sum over a list of 16-bit LDS slots (eight entries per chunk) of a
// neighborhood copy at LDS address 0: half
// the bytes of the 32-bit list per entry.  The body covers two chunks, with
// the same look-ahead discipline (index chunks one to two chunks ahead,
// positions two entries ahead, unconditional memory operations, the chunk
// after the last standing in for every chunk past the end).  With L lanes
// per atom, lane p of the group walks chunks p, p + L, p + 2L, ...  The
// caller passes the lane's first two chunks (p and p + L, at most row 7),
// which every 16-bit list fills (with sentinels past the count), so it can
// load them before the count is known.  The only exit
// is at the end of the body: a loop with several exits loses the exact wait
// counts at its head.
template <bool THERMO, int IMG, bool HALF = false>
__device__ __forceinline__ void pair_sum16(const v4i *__restrict__ chunks, v4i i0, v4i i1, int p, int L, int c,
                                           double xi, double yi, double zi, const Box &B, double mf6, double mu6,
                                           double &ax, double &ay, double &az, double &u, double &w,
                                           lds_double *R = nullptr, int s_lo = 0) {
    const int nch = (c + 7) >> 3;
    // this lane's k-th chunk is chunk p + L k of the atom's list
    auto ld = [&](int k) {
        const int q = p + L * k;
        return __builtin_nontemporal_load(chunks + (q < nch ? q : nch) * 64);
    };
    // a half list's words keep their marks for the evaluation; the slots
    // drop them for the address
    Duo P_, Q_;
    unsigned wP = 0u, wQ = 0u;
    auto fetchP = [&](int word) {
        wP = unsigned(word);
        fetch2w(HALF ? int(unsigned(word) & 0x7FFF7FFFu) : word, P_);
    };
    auto fetchQ = [&](int word) {
        wQ = unsigned(word);
        fetch2w(HALF ? int(unsigned(word) & 0x7FFF7FFFu) : word, Q_);
    };
    auto evalP = [&]() { eval2<THERMO, IMG, HALF>(P_, xi, yi, zi, B, mf6, mu6, ax, ay, az, u, w, wP, R, s_lo); };
    auto evalQ = [&]() { eval2<THERMO, IMG, HALF>(Q_, xi, yi, zi, B, mf6, mu6, ax, ay, az, u, w, wQ, R, s_lo); };
    fetchP(i0[0]);
    int k = 0;
    for (;; k += 2) {
        fetchQ(i0[1]);
        evalP();
        fetchP(i0[2]);
        evalQ();
        fetchQ(i0[3]);
        evalP();
        fetchP(i1[0]);
        i0 = ld(k + 2);
        evalQ();
        fetchQ(i1[1]);
        evalP();
        fetchP(i1[2]);
        evalQ();
        fetchQ(i1[3]);
        evalP();
        fetchP(i0[0]);
        i1 = ld(k + 3);
        evalQ();
        if (!__any(p + L * (k + 3) < nch))
            break;
    }
    // fewer than two of the lane's chunks remain: the first of them (in i0,
    // its first two positions in P) runs here if any lane still has it, so
    // an odd chunk count does not cost a chunk of sentinels
    if (__any(p + L * (k + 2) < nch)) {
        fetchQ(i0[1]);
        evalP();
        fetchP(i0[2]);
        evalQ();
        fetchQ(i0[3]);
        evalP();
        evalQ();
    }
    __builtin_amdgcn_s_waitcnt(0x0070);  // vmcnt(0) expcnt(7) lgkmcnt(0)
}

__device__ __forceinline__ const v4i *list_chunks(const int32_t *nbr, int i, int nchunk) {
    return reinterpret_cast<const v4i *>(nbr) + (int64_t(i >> 6) * nchunk) * 64 + (i & 63);
}

// The end of an atom's step in the force kernels, given its force a: MODE
// 0 stores F, 1 stores F and kicks v += h F, 2 kicks twice and drifts into
// the other position buffer (k_force's epilogue).
template <int MODE, bool THERMO>
__device__ __forceinline__ void atom_epilogue(const Dims &d, int i, double xi, double yi, double zi, double ax,
                                              double ay, double az, const Box &B, double *vx, double *vy, double *vz,
                                              double *fx, double *fy, double *fz, double *pout, double &ke,
                                              int32_t *err) {
    if (MODE == 0 || MODE == 1) {
        fx[i] = ax;
        fy[i] = ay;
        fz[i] = az;
        if (!(isfinite(ax) && isfinite(ay) && isfinite(az)))
            atomicOr(err, kErrNonFinite);
    }
    if (MODE >= 1) {
        double a = vx[i] + B.h * ax, bb = vy[i] + B.h * ay, c = vz[i] + B.h * az;
        if (THERMO)
            ke += a * a + bb * bb + c * c;
        if (MODE == 2) {
            a = a + B.h * ax;
            bb = bb + B.h * ay;
            c = c + B.h * az;
            const double nx = xi + B.dt * a, ny = yi + B.dt * bb, nz = zi + B.dt * c;
            pos_put(d.layout, d.ntp, pout, i, nx, ny, nz);
            if (!(isfinite(nx) && isfinite(ny) && isfinite(nz)))
                atomicOr(err, kErrNonFinite);
        }
        vx[i] = a;
        vy[i] = bb;
        vz[i] = c;
    }
}

// One workgroup per block, one lane per atom.  MODE 0: store F.  MODE 1:
// store F and kick v += h F.  MODE 2: kick twice (closing this step and
// opening the next) and drift into the other position buffer.  With THERMO
// each block writes its partial sums of the pair energy, of s f(s) and of
// |v|^2 at the full step - no atomics anywhere.
// HALF (L = 1, one workgroup per block): the lists are half lists inside
// half-list blocks (block_half()); there each atom's own sum and its
// partners' reactions meet in LDS sums over the own cells' slot span, and
// after a barrier every atom takes its total and finishes the step.  Those
// sums are LDS atomics, so their order - and the last bits of the forces -
// may vary from run to run.  Other blocks finish each atom directly.
template <int MODE, bool THERMO, int L, bool HALF = false>
__global__ __launch_bounds__(kMaxThreads) void k_force(Dims d, const Box *__restrict__ boxes,
                                                       const int32_t *__restrict__ blk_box,
                                                       const double *__restrict__ pin,
                                                       const int32_t *__restrict__ hood_tab,
                                                       const int32_t *__restrict__ cnt,
                                                       const int32_t *__restrict__ nbr, double *__restrict__ vx,
                                                       double *__restrict__ vy, double *__restrict__ vz,
                                                       double *__restrict__ fx, double *__restrict__ fy,
                                                       double *__restrict__ fz, double *__restrict__ pout,
                                                       double *__restrict__ partials, int32_t *err) {
    // no static LDS: the neighborhood copy starts at LDS address 0, where
    // the pair loop's slot addresses point, and the table and reduction
    // scratch follow it
    extern __shared__ double lds[];
    const int tail = (d.cap + 2 + kHoodPad) * 24;
    Hood &h = *reinterpret_cast<Hood *>(reinterpret_cast<char *>(lds) + tail);
    double(*red)[kMaxThreads / 64] =
        reinterpret_cast<double(*)[kMaxThreads / 64]>(reinterpret_cast<char *>(lds) + tail + kHoodBytes8);
    int b, part;
    if (!block_part(d, b, part))
        return;
    // the prologue (table, staging) waits on memory while the other
    // workgroup on the CU runs its pair loop: its waves issue first, so the
    // loads go out early, and drop back to normal priority for the loop
    __builtin_amdgcn_s_setprio(2);
    if (threadIdx.x == 0 && unsigned(uintptr_t((lds_char *)lds)) != 0u)
        atomicOr(err, kErrLdsLayout);
    HoodWords hw;
    hood_fetch(hood_tab, b, hw);
    const Box B = block_box(d, boxes, blk_box, b);
    // -f6 and -u6 live in vector registers: each fma of the pair loop that
    // uses them already reads one scalar operand
    double mf6 = -B.f6, mu6 = -B.u6;
    asm volatile("" : "+v"(mf6), "+v"(mu6));
    hood_commit(hw, h);
    const int total = h.off[h.ncell];
    const bool fits = total <= d.cap;
    lds_double *const S = (lds_double *)lds;
    const GlobalPos gpos{pos_of(d.layout, d.ntp, pin)};
    const HoodImage im = hood_image(B, b - B.block_off, fits);
    // half lists: the reaction sums follow the table and reduction scratch
    lds_double *R = (lds_double *)((lds_char *)lds + tail + kForceLdsTail);
    int s_lo = 0, span = 0;
    const bool half = HALF && block_half(d, B, b - B.block_off, h, fits, s_lo, span);
    if (HALF && half)
        for (int k = threadIdx.x; k < 3 * span; k += blockDim.x)
            R[k] = 0.0;  // the staging ends with a barrier
    // The operands of a lane's next atom (position, list length, velocity)
    // are loaded one pass ahead - those of the first pass before the staging
    // barrier, so their latency overlaps the staging.  Past the block's last
    // atom the loads read that atom again (a cache hit) and are not used.
    // L lanes per atom (adjacent lanes), lane p of the group taking every
    // L-th chunk of the list; their sums are combined before the epilogue
    const int p = threadIdx.x & (L - 1);
    const int T = blockDim.x / L;
    int lo, hi;
    h.share(part, d.parts, lo, hi);
    int i = lo + threadIdx.x / L;
    double xi = 0.0, yi = 0.0, zi = 0.0, vxi = 0.0, vyi = 0.0, vzi = 0.0;
    int ci = 0;
    v4i r0 = {0, 0, 0, 0}, r1 = {0, 0, 0, 0};
    auto load_atom = [&](int k) {
        const int ic = min(k, hi - 1);
        pos_get(d.layout, d.ntp, pin, ic, xi, yi, zi);
        ci = cnt[ic];
        if (MODE >= 1) {
            vxi = vx[ic];
            vyi = vy[ic];
            vzi = vz[ic];
        }
        if (fits) {  // this lane's first two rows (p and p + L) of the 16-bit list
            // (a row past the atom's area stands for a chunk past the end of
            // the list: the area's last row is then sentinel padding)
            const v4i *ch = list_chunks(nbr, ic, d.nchunk);
            r0 = __builtin_nontemporal_load(ch + min(p, d.nchunk - 1) * 64);
            r1 = __builtin_nontemporal_load(ch + min(p + L, d.nchunk - 1) * 64);
        }
    };
    if (hi > lo)
        load_atom(i);
    if (fits)
        hood_stage(h, total, d.cap, pos_of(d.layout, d.ntp, pin), S, im);
    // have every kernel argument in registers before the atom loop: a scalar
    // load still in flight at the pair loop's head costs it exact LDS waits
    asm volatile("" ::"s"(err), "s"(partials), "s"(pout), "s"(fx));
    __builtin_amdgcn_s_setprio(0);
    double u = 0.0, w = 0.0, ke = 0.0;
    for (; i < hi; i += T) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        const v4i *chunks = list_chunks(nbr, i, d.nchunk);
        if (im.on && !im.check)
            pair_sum16<THERMO, 1, HALF>(chunks, r0, r1, p, L, ci, xi, yi, zi, B, mf6, mu6, ax, ay, az, u, w, R,
                                        s_lo);
        else if (im.on)
            pair_sum16<THERMO, 2, HALF>(chunks, r0, r1, p, L, ci, xi, yi, zi, B, mf6, mu6, ax, ay, az, u, w, R,
                                        s_lo);
        else if (fits)
            pair_sum16<THERMO, 0, HALF>(chunks, r0, r1, p, L, ci, xi, yi, zi, B, mf6, mu6, ax, ay, az, u, w, R,
                                        s_lo);
        else
            pair_sum<THERMO>(chunks, p, L, ci, gpos, xi, yi, zi, B, mf6, mu6, ax, ay, az, u, w);
        // combine the L partial sums of the group (a butterfly: addition
        // commutes, so every lane of the group ends with the same bits)
#pragma unroll
        for (int o = 1; o < L; o <<= 1) {
            ax += __shfl_xor(ax, o, 64);
            ay += __shfl_xor(ay, o, 64);
            az += __shfl_xor(az, o, 64);
        }
        const bool own = p == 0;  // the group's first lane writes the atom
        if (HALF && half) {
            lds_double *r = R + 3 * (own_slot(B, b - B.block_off, h, i) - s_lo);
            __hip_atomic_fetch_add((double *)r, ax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add((double *)(r + 1), ay, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add((double *)(r + 2), az, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            load_atom(i + T);
            continue;
        }
        if ((MODE == 0 || MODE == 1) && own) {
            fx[i] = ax;
            fy[i] = ay;
            fz[i] = az;
            if (!(isfinite(ax) && isfinite(ay) && isfinite(az)))
                atomicOr(err, kErrNonFinite);
        }
        if (MODE >= 1 && own) {
            double a = vxi + B.h * ax, bb = vyi + B.h * ay, c = vzi + B.h * az;
            if (THERMO)
                ke += a * a + bb * bb + c * c;
            if (MODE == 2) {
                a = a + B.h * ax;
                bb = bb + B.h * ay;
                c = c + B.h * az;
                // not wrapped: between list builds an atom stays next to its
                // block's cells (the binning wraps)
                const double nx = xi + B.dt * a, ny = yi + B.dt * bb, nz = zi + B.dt * c;
                pos_put(d.layout, d.ntp, pout, i, nx, ny, nz);
                if (!(isfinite(nx) && isfinite(ny) && isfinite(nz)))
                    atomicOr(err, kErrNonFinite);
            }
            vx[i] = a;
            vy[i] = bb;
            vz[i] = c;
        }
        load_atom(i + T);
    }
    if (HALF && half) {
        __syncthreads();
        for (int k = lo + threadIdx.x; k < hi; k += blockDim.x) {
            const lds_double *r = R + 3 * (own_slot(B, b - B.block_off, h, k) - s_lo);
            double xk, yk, zk;
            pos_get(d.layout, d.ntp, pin, k, xk, yk, zk);
            atom_epilogue<MODE, THERMO>(d, k, xk, yk, zk, r[0], r[1], r[2], B, vx, vy, vz, fx, fy, fz, pout, ke, err);
        }
    }
    if (THERMO) {
        block_sum3(u, w, ke, red);
        if (threadIdx.x == 0) {
            const int q = b * d.parts + part;
            partials[q * kPartialStride + 0] = u;
            partials[q * kPartialStride + 1] = w;
            partials[q * kPartialStride + 2] = ke;
        }
    }
}

// First half of a step when F of the current positions is already stored.
__global__ __launch_bounds__(kAtomThreads) void k_drift(Dims d, const Box *__restrict__ boxes,
                                                        const int32_t *__restrict__ atom_box,
                                                        const double *__restrict__ pin, double *__restrict__ vx,
                                                        double *__restrict__ vy, double *__restrict__ vz,
                                                        const double *__restrict__ fx,
                                                        const double *__restrict__ fy,
                                                        const double *__restrict__ fz, double *__restrict__ pout,
                                                        int32_t *err) {
    const int i = blockIdx.x * kAtomThreads + threadIdx.x;
    if (i >= d.nt)
        return;
    const Box &B = boxes[atom_box[i]];
    const double a = vx[i] + B.h * fx[i], b = vy[i] + B.h * fy[i], c = vz[i] + B.h * fz[i];
    vx[i] = a;
    vy[i] = b;
    vz[i] = c;
    double px, py, pz;
    pos_get(d.layout, d.ntp, pin, i, px, py, pz);
    const double nx = px + B.dt * a, ny = py + B.dt * b, nz = pz + B.dt * c;  // wrapped at binning
    pos_put(d.layout, d.ntp, pout, i, nx, ny, nz);
    if (!(isfinite(nx) && isfinite(ny) && isfinite(nz)))
        atomicOr(err, kErrNonFinite);
}

// One wavefront per box sums that box's workgroup partials (parts per
// block) in a fixed order.
__global__ __launch_bounds__(64) void k_reduce(const Box *__restrict__ boxes, const double *__restrict__ partials,
                                               int parts, double *out, int row_len) {
    const Box &B = boxes[blockIdx.x];
    double u = 0.0, w = 0.0, k = 0.0;
    for (int q = threadIdx.x; q < B.nblocks * parts; q += 64) {
        const int blk = B.block_off * parts + q;
        u += partials[blk * kPartialStride + 0];
        w += partials[blk * kPartialStride + 1];
        k += partials[blk * kPartialStride + 2];
    }
    u = wave_sum(u);
    w = wave_sum(w);
    k = wave_sum(k);
    if (threadIdx.x == 0) {
        const double U = 0.5 * u, W = 0.5 * w, KE = 0.5 * B.mass * k;
        double *row = out + int64_t(blockIdx.x) * row_len;
        if (row_len == 2) {
            row[0] = U;
            row[1] = W;
        } else {
            row[0] = KE;
            row[1] = B.n > 1 ? 2.0 * KE / (3.0 * B.n - 3.0) : 0.0;
            row[2] = U;
            row[3] = W;
            row[4] = KE + U;
        }
    }
}

// Current list in original ids, rows sorted ascending, unused slots -1.
__global__ __launch_bounds__(kMaxThreads) void k_export_neighbors(Dims d, const Box *__restrict__ boxes,
                                                                  const int32_t *__restrict__ blk_box,
                                                                  const int32_t *__restrict__ cell_start,
                                                                  const int32_t *__restrict__ cnt,
                                                                  const int32_t *__restrict__ nbr,
                                                                  const int32_t *__restrict__ orig,
                                                                  int32_t *counts, int32_t *ids) {
    __shared__ Hood h;
    const int b = xcd_remap();
    if (b >= d.nblk)
        return;
    const Box B = block_box(d, boxes, blk_box, b);
    hood_setup(B, b - B.block_off, cell_start, h);
    const bool fits = h.off[h.ncell] <= d.cap;
    const uint16_t *nbr16 = reinterpret_cast<const uint16_t *>(nbr);
    for (int i = h.a0 + threadIdx.x; i < h.a1; i += blockDim.x) {
        const int o = orig[i], c = cnt[i];
        counts[o] = c;
        if (!ids)
            continue;
        int32_t *row = ids + int64_t(o) * d.maxnb;
        for (int k = 0; k < c; ++k) {
            // (bit 15 of a 16-bit entry marks a half-list pair inside the block)
            int g = fits ? int(nbr16[nbr_index16(i, k, d.nchunk)] & 0x7FFFu) : nbr[nbr_index(i, k, d.nchunk)];
            if (fits) {
                const int uu = hood_find(h, g);
                g = h.cs[uu] + (g - h.off[uu]);
            }
            const int v = orig[g];
            int q = k - 1;
            while (q >= 0 && row[q] > v) {
                row[q + 1] = row[q];
                --q;
            }
            row[q + 1] = v;
        }
        for (int k = c; k < d.maxnb; ++k)
            row[k] = -1;
    }
}

// ------------------------------------------------------------------ adjoint

// Neighborhood staged with positions and one vector field w: 48 bytes per
// LDS slot (x, y, z, wx, wy, wz); the sentinel slot has NaN positions.
__device__ __forceinline__ lds_double *lds_slot6(lds_double *base, int slot) {
    return (lds_double *)((lds_char *)base + __umul24(unsigned(slot), 48u));
}

__device__ __forceinline__ void hood_stage6(const Hood &h, int total, int sent, const Pos &x, const Pos &w,
                                            lds_double *s, const HoodImage &im) {
    // as hood_stage: four slots per thread per round, unconditional memory
    // operations, a slot past the end copied into the scratch slot sent + 1
    constexpr int R = 4;
    const int T = blockDim.x;
    for (int base = threadIdx.x; base < total; base += R * T) {
        int ts[R], us[R], g[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            ts[r] = min(base + r * T, total - 1);
        hood_find_n<R>(h, ts, us);
#pragma unroll
        for (int r = 0; r < R; ++r)
            g[r] = h.cs[us[r]] + (ts[r] - h.off[us[r]]);
        double v[R][6];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v[r][0] = x.x[g[r]];
            v[r][1] = x.y[g[r]];
            v[r][2] = x.z[g[r]];
            v[r][3] = w.x[g[r]];
            v[r][4] = w.y[g[r]];
            v[r][5] = w.z[g[r]];
        }
        if (im.on) {  // the force kernel's images (same positions, same shifts)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                v[r][0] = nearest_image(v[r][0], im.cx, im.L, im.halfL);
                v[r][1] = nearest_image(v[r][1], im.cy, im.L, im.halfL);
                v[r][2] = nearest_image(v[r][2], im.cz, im.L, im.halfL);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            lds_double *a = lds_slot6(s, base + r * T < total ? base + r * T : sent + 1);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                a[k] = v[r][k];
        }
    }
    if (threadIdx.x == 0) {
        lds_double *a = lds_slot6(s, sent);
        a[0] = a[1] = a[2] = __builtin_nan("");
        a[3] = a[4] = a[5] = 0.0;
    }
    __syncthreads();
}

// Positions and w of two list entries.
struct Duo6 {
    double x[2], y[2], z[2], wx[2], wy[2], wz[2];
};

__device__ __forceinline__ void fetch2w6(lds_double *S, int word, Duo6 &q) {
    const unsigned wd = unsigned(word);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const lds_double *a = lds_slot6(S, int(m == 0 ? (wd & 0xffffu) : (wd >> 16)));
        q.x[m] = a[0];
        q.y[m] = a[1];
        q.z[m] = a[2];
        q.wx[m] = a[3];
        q.wy[m] = a[4];
        q.wz[m] = a[5];
    }
}

// Constants of the reverse pair terms that live in vector registers (each
// fma that uses them already reads one scalar operand).
struct HvpConst {
    double mf6, me6, mh6, g8;
};

// Reverse-mode terms of one pair (the cutoff decision is the force kernel's:
// same geometry, same fused |d|^2):
//   (J w)_i += f(s) u + 2 f'(s) (d . u) d,  u = w_i - w_j,
//   pe += (df/deps) (w_i . d),  ps += (df/dsigma) (w_i . d),
// with q = sr2^3, f = sr2 q (f12 q - f6), 2 f' = sr2^2 q (g8 - g14 q),
// df/deps = sr2 q (e12 q - e6), df/dsigma = sr2 q (h12 q - h6).  IMG as in
// eval2.
template <int IMG>
__device__ __forceinline__ void hvp_pair(double xj, double yj, double zj, double wxj, double wyj, double wzj,
                                         double xi, double yi, double zi, double wxi, double wyi, double wzi,
                                         const Box &B, const HvpConst &k, double &gx, double &gy, double &gz,
                                         double &pe, double &ps) {
    double dx, dy, dz;
    const double s = pair_geom<IMG>(xi, yi, zi, xj, yj, zj, B, dx, dy, dz);
    if (s < B.rc2) {
        const double sr2 = recip_exact(s);
        const double q3 = sr2 * sr2 * sr2;
        const double a = sr2 * q3;
        const double f = a * fma(B.f12, q3, k.mf6);
        const double fe = a * fma(B.e12, q3, k.me6);
        const double fs = a * fma(B.h12, q3, k.mh6);
        const double c2 = (sr2 * a) * fma(-B.g14, q3, k.g8);
        const double ux = wxi - wxj, uy = wyi - wyj, uz = wzi - wzj;
        const double t2 = c2 * fma(dz, uz, fma(dy, uy, dx * ux));
        gx = fma(f, ux, fma(t2, dx, gx));
        gy = fma(f, uy, fma(t2, dy, gy));
        gz = fma(f, uz, fma(t2, dz, gz));
        const double wd = fma(wzi, dz, fma(wyi, dy, wxi * dx));
        pe = fma(fe, wd, pe);
        ps = fma(fs, wd, ps);
    }
}

// hvp terms over a 16-bit list, with pair_sum16's loop discipline and its
// split of the list over L lanes per atom (lane p walks chunks p, p + L,
// ...; i0 and i1 are the lane's first two chunks).
template <int IMG>
__device__ __forceinline__ void hvp_sum16(const v4i *__restrict__ chunks, v4i i0, v4i i1, int p, int L, int c,
                                          lds_double *S, double xi, double yi, double zi, double wxi, double wyi,
                                          double wzi, const Box &B, const HvpConst &k, double &gx, double &gy,
                                          double &gz, double &pe, double &ps) {
    const int nch = (c + 7) >> 3;
    auto ld = [&](int kk) {
        const int q = p + L * kk;
        return __builtin_nontemporal_load(chunks + (q < nch ? q : nch) * 64);
    };
    auto ev = [&](const Duo6 &q) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
            hvp_pair<IMG>(q.x[m], q.y[m], q.z[m], q.wx[m], q.wy[m], q.wz[m], xi, yi, zi, wxi, wyi, wzi, B, k, gx, gy,
                          gz, pe, ps);
    };
    Duo6 P, Q;
    fetch2w6(S, i0[0], P);
    int kk = 0;
    for (;; kk += 2) {
        fetch2w6(S, i0[1], Q);
        ev(P);
        fetch2w6(S, i0[2], P);
        ev(Q);
        fetch2w6(S, i0[3], Q);
        ev(P);
        fetch2w6(S, i1[0], P);
        i0 = ld(kk + 2);
        ev(Q);
        fetch2w6(S, i1[1], Q);
        ev(P);
        fetch2w6(S, i1[2], P);
        ev(Q);
        fetch2w6(S, i1[3], Q);
        ev(P);
        fetch2w6(S, i0[0], P);
        i1 = ld(kk + 3);
        ev(Q);
        if (!__any(p + L * (kk + 3) < nch))
            break;
    }
    if (__any(p + L * (kk + 2) < nch)) {  // an odd last chunk, as in pair_sum16
        fetch2w6(S, i0[1], Q);
        ev(P);
        fetch2w6(S, i0[2], P);
        ev(Q);
        fetch2w6(S, i0[3], Q);
        ev(P);
        ev(Q);
    }
    __builtin_amdgcn_s_waitcnt(0x0070);  // vmcnt(0) expcnt(7) lgkmcnt(0)
}

// Reverse-mode step at one force evaluation of the velocity-Verlet map,
// with the list and the cutoff indicators of the forward run held fixed.
// For w = lam_v (one lane per atom, one workgroup per block):
//   (J w)_i = sum_{j in list(i), s < rc^2} [ f(s) (w_i - w_j) + 2 f'(s) ((w_i - w_j) . d_ij) d_ij ]
// (the terms of hvp_pair); lam_x_i += c (J w)_i, c = mult * dt / (2 m).  The
// workgroup adds mult times its partial sums of w_i . dF_i/deps and
// w_i . dF_i/dsigma to its slot of `partials` (which the reverse sweep
// clears first and reduces over each box's blocks once, at its end).  With drift_adj the adjoint of the drift before this force
// evaluation follows: wout_i = w_i + dt lam_x_i.  The neighborhood is staged
// with w (48 bytes per slot).  L lanes per atom split its list as the force
// kernel's lanes do (groups of eight entries dealt in turn, on the 32-bit
// path too, so both paths give the same sums) and combine their sums by a
// butterfly; the atom's first lane writes.
// (at most kHvpThreads threads: its 48-byte LDS slots leave room for one
// workgroup per CU at the usual capacities, so the bound costs no occupancy
// and lets the compiler keep the 2- and 4-lane variants' registers out of
// scratch memory)
constexpr int kHvpThreads = 768;

template <int L>
__global__ __launch_bounds__(kHvpThreads) void k_hvp(Dims d, const Box *__restrict__ boxes,
                                                     const int32_t *__restrict__ blk_box, Pos x,
                                                     const int32_t *__restrict__ hood_tab,
                                                     const int32_t *__restrict__ cnt,
                                                     const int32_t *__restrict__ nbr, Pos w, Pos lam, Pos wout,
                                                     double mult, int drift_adj, double *__restrict__ partials) {
    __shared__ Hood h;
    extern __shared__ double lds[];
    int b, part;
    if (!block_part(d, b, part))
        return;
    HoodWords hw;
    hood_fetch(hood_tab, b, hw);
    const Box B = block_box(d, boxes, blk_box, b);
    HvpConst k{-B.f6, -B.e6, -B.h6, B.g8};
    asm volatile("" : "+v"(k.mf6), "+v"(k.me6), "+v"(k.mh6), "+v"(k.g8));
    hood_commit(hw, h);
    const int total = h.off[h.ncell];
    const bool fits = total <= d.cap;
    lds_double *S = (lds_double *)lds;
    const HoodImage im = hood_image(B, b - B.block_off, fits);
    if (fits)
        hood_stage6(h, total, d.cap, x, w, S, im);
    asm volatile("" ::"s"(partials), "s"(wout.x), "s"(lam.x));
    double pe = 0.0, ps = 0.0, unused = 0.0;
    int lo, hi;
    h.share(part, d.parts, lo, hi);
    const int p = threadIdx.x & (L - 1);
    const int T = blockDim.x / L;
    for (int i = lo + threadIdx.x / L; i < hi; i += T) {
        const double xi = x.x[i], yi = x.y[i], zi = x.z[i];
        const double wxi = w.x[i], wyi = w.y[i], wzi = w.z[i];
        double gx = 0.0, gy = 0.0, gz = 0.0;
        const int c = cnt[i];
        const v4i *chunks = list_chunks(nbr, i, d.nchunk);
        if (fits) {
            // rows p and p + L (at most row 7): every 16-bit list fills them
            const v4i r0 = __builtin_nontemporal_load(chunks + min(p, d.nchunk - 1) * 64);
            const v4i r1 = __builtin_nontemporal_load(chunks + min(p + L, d.nchunk - 1) * 64);
            if (im.on && !im.check)
                hvp_sum16<1>(chunks, r0, r1, p, L, c, S, xi, yi, zi, wxi, wyi, wzi, B, k, gx, gy, gz, pe, ps);
            else if (im.on)
                hvp_sum16<2>(chunks, r0, r1, p, L, c, S, xi, yi, zi, wxi, wyi, wzi, B, k, gx, gy, gz, pe, ps);
            else
                hvp_sum16<0>(chunks, r0, r1, p, L, c, S, xi, yi, zi, wxi, wyi, wzi, B, k, gx, gy, gz, pe, ps);
        } else {
            // groups of eight entries dealt in turn, as on the 16-bit path;
            // past the count the 32-bit list holds sentinels (global slot nt)
            // through the chunk after its last one, which add nothing
            const int ng = (c + 7) >> 3;
            for (int g = p; g < ng; g += L)
                for (int e = 0; e < 8; ++e) {
                    const int j = nbr[nbr_index(i, 8 * g + e, d.nchunk)];
                    hvp_pair<0>(x.x[j], x.y[j], x.z[j], w.x[j], w.y[j], w.z[j], xi, yi, zi, wxi, wyi, wzi, B, k,
                                    gx, gy, gz, pe, ps);
                }
        }
#pragma unroll
        for (int o = 1; o < L; o <<= 1) {
            gx += __shfl_xor(gx, o, 64);
            gy += __shfl_xor(gy, o, 64);
            gz += __shfl_xor(gz, o, 64);
        }
        if (p != 0)
            continue;
        const double cc = mult * B.h;
        const double lx = lam.x[i] + cc * gx, ly = lam.y[i] + cc * gy, lz = lam.z[i] + cc * gz;
        lam.x[i] = lx;
        lam.y[i] = ly;
        lam.z[i] = lz;
        if (drift_adj) {
            wout.x[i] = wxi + B.dt * lx;
            wout.y[i] = wyi + B.dt * ly;
            wout.z[i] = wzi + B.dt * lz;
        }
    }
    block_sum3(pe, ps, unused);
    if (threadIdx.x == 0) {
        double *q = partials + (b * d.parts + part) * kPartialStride;
        q[0] += mult * pe;
        q[1] += mult * ps;
    }
}

// ------------------------------------------------------------------ Spring-Dashpot

// One Spring-Dashpot pair term (Sec. 3.2, Eq. 3) on sphere i: while the
// spheres overlap (r < sigma), F_ij = [K (sigma - r) - gamma (u . v_ij)] u
// with u = x_ij / r and v_ij = v_i - v_j; with THERMO the elastic energy
// K (sigma - r)^2 / 2 and x_ij . F_ij = r times the magnitude.  A NaN
// sentinel entry fails the overlap test.  IMG as in eval2.
template <bool THERMO, int IMG>
__device__ __forceinline__ void sd_term(double xj, double yj, double zj, double vxj, double vyj, double vzj,
                                        double xi, double yi, double zi, double vxi, double vyi, double vzi,
                                        const Box &B, double &ax, double &ay, double &az, double &u, double &w) {
    double dx, dy, dz;
    const double s = pair_geom<IMG>(xi, yi, zi, xj, yj, zj, B, dx, dy, dz);
    if (s < B.sd_sig2) {
        const double r = sqrt(s);
        const double ir = 1.0 / r;
        const double ux = dx * ir, uy = dy * ir, uz = dz * ir;
        const double un = fma(uz, vzi - vzj, fma(uy, vyi - vyj, ux * (vxi - vxj)));
        const double ov = B.sd_sig - r;
        const double fm = fma(B.sd_k, ov, -(B.sd_g * un));
        ax = fma(fm, ux, ax);
        ay = fma(fm, uy, ay);
        az = fma(fm, uz, az);
        if (THERMO) {
            u = fma(0.5 * B.sd_k * ov, ov, u);
            w = fma(fm, r, w);
        }
    }
}

// Spring-Dashpot force on every sphere of a block, one lane per sphere, the
// neighborhood staged with velocities (48 bytes a slot); MODE and the
// epilogue as in k_force, except that kicked velocities go to vo, another
// buffer than v.  The velocities read are those stored when the kernel runs
// - the half-step velocities inside an integration, the initial ones at the
// first force.
template <int MODE, bool THERMO>
__global__ __launch_bounds__(kMaxThreads) void k_force_sd(Dims d, const Box *__restrict__ boxes,
                                                          const int32_t *__restrict__ blk_box, Pos x,
                                                          const int32_t *__restrict__ hood_tab,
                                                          const int32_t *__restrict__ cnt,
                                                          const int32_t *__restrict__ nbr, Pos v, Pos vo, Pos f,
                                                          Pos xo, double *__restrict__ partials, int32_t *err) {
    __shared__ Hood h;
    extern __shared__ double lds[];
    int b, part;
    if (!block_part(d, b, part))
        return;
    HoodWords hw;
    hood_fetch(hood_tab, b, hw);
    const Box B = block_box(d, boxes, blk_box, b);
    hood_commit(hw, h);
    const int total = h.off[h.ncell];
    const bool fits = total <= d.cap;
    lds_double *S = (lds_double *)lds;
    const HoodImage im = hood_image(B, b - B.block_off, fits);
    if (fits)
        hood_stage6(h, total, d.cap, x, v, S, im);
    double u = 0.0, w = 0.0, ke = 0.0;
    int lo, hi;
    h.share(part, d.parts, lo, hi);
    const uint16_t *nbr16 = reinterpret_cast<const uint16_t *>(nbr);
    for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double xi = x.x[i], yi = x.y[i], zi = x.z[i];
        const double vxi = v.x[i], vyi = v.y[i], vzi = v.z[i];
        const int c = cnt[i];
        double ax = 0.0, ay = 0.0, az = 0.0;
        if (fits) {
            for (int k = 0; k < c; ++k) {
                const lds_double *a = lds_slot6(S, nbr16[nbr_index16(i, k, d.nchunk)]);
                if (im.on && !im.check)
                    sd_term<THERMO, 1>(a[0], a[1], a[2], a[3], a[4], a[5], xi, yi, zi, vxi, vyi, vzi, B, ax, ay, az,
                                       u, w);
                else if (im.on)
                    sd_term<THERMO, 2>(a[0], a[1], a[2], a[3], a[4], a[5], xi, yi, zi, vxi, vyi, vzi, B, ax, ay, az,
                                       u, w);
                else
                    sd_term<THERMO, 0>(a[0], a[1], a[2], a[3], a[4], a[5], xi, yi, zi, vxi, vyi, vzi, B, ax, ay, az,
                                       u, w);
            }
        } else {
            for (int k = 0; k < c; ++k) {
                const int j = nbr[nbr_index(i, k, d.nchunk)];
                sd_term<THERMO, 0>(x.x[j], x.y[j], x.z[j], v.x[j], v.y[j], v.z[j], xi, yi, zi, vxi, vyi, vzi, B,
                                       ax, ay, az, u, w);
            }
        }
        if (MODE == 0 || MODE == 1) {
            f.x[i] = ax;
            f.y[i] = ay;
            f.z[i] = az;
            if (!(isfinite(ax) && isfinite(ay) && isfinite(az)))
                atomicOr(err, kErrNonFinite);
        }
        if (MODE >= 1) {
            double va = vxi + B.h * ax, vb = vyi + B.h * ay, vc = vzi + B.h * az;
            if (THERMO)
                ke += va * va + vb * vb + vc * vc;
            if (MODE == 2) {
                va = va + B.h * ax;
                vb = vb + B.h * ay;
                vc = vc + B.h * az;
                const double nx = xi + B.dt * va, ny = yi + B.dt * vb, nz = zi + B.dt * vc;
                xo.x[i] = nx;
                xo.y[i] = ny;
                xo.z[i] = nz;
                if (!(isfinite(nx) && isfinite(ny) && isfinite(nz)))
                    atomicOr(err, kErrNonFinite);
            }
            // (another half than v: other workgroups still read this
            // sphere's velocity as a neighbour's)
            vo.x[i] = va;
            vo.y[i] = vb;
            vo.z[i] = vc;
        }
    }
    if (THERMO) {
        block_sum3(u, w, ke);
        if (threadIdx.x == 0) {
            const int q = b * d.parts + part;
            partials[q * kPartialStride + 0] = u;
            partials[q * kPartialStride + 1] = w;
            partials[q * kPartialStride + 2] = ke;
        }
    }
}

// acc[2 box + q] += mult * h * (sum over the box's blocks of partial q), one
// wavefront per box, fixed order (the reverse sweep's partials hold the sums
// over all of its steps: it calls this once, with mult 1).
__global__ __launch_bounds__(64) void k_grad_reduce(const Box *__restrict__ boxes,
                                                    const double *__restrict__ partials, int parts, double mult,
                                                    double *acc) {
    const Box &B = boxes[blockIdx.x];
    double e = 0.0, s = 0.0;
    for (int q = threadIdx.x; q < B.nblocks * parts; q += 64) {
        const int blk = B.block_off * parts + q;
        e += partials[blk * kPartialStride + 0];
        s += partials[blk * kPartialStride + 1];
    }
    e = wave_sum(e);
    s = wave_sum(s);
    if (threadIdx.x == 0) {
        acc[2 * blockIdx.x] += mult * B.h * e;
        acc[2 * blockIdx.x + 1] += mult * B.h * s;
    }
}

__global__ __launch_bounds__(kAtomThreads) void k_gather(int n, const double *__restrict__ s0,
                                                         const double *__restrict__ s1,
                                                         const double *__restrict__ s2,
                                                         const int32_t *__restrict__ orig, Pos dst) {
    const int p = blockIdx.x * kAtomThreads + threadIdx.x;
    if (p >= n)
        return;
    const int o = orig[p];
    dst.x[p] = s0 ? s0[o] : 0.0;
    dst.y[p] = s1 ? s1[o] : 0.0;
    dst.z[p] = s2 ? s2[o] : 0.0;
}

__global__ void k_fill_f64(double *p, double v, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

// One box descriptor written from a kernel argument (no host staging copy).
__global__ void k_store_box(Box *dst, Box B) {
    if (threadIdx.x == 0)
        *dst = B;
}

// The device error word as a status code (the codes tmd_sync returns):
// out[0] = status, out[1] = largest list length requested on overflow.
__global__ void k_status_out(const int32_t *__restrict__ err, int32_t *out) {
    if (threadIdx.x != 0)
        return;
    const int w = err[0];
    int st = 0;
    if (w & kErrNonFinite)
        st = -5;
    else if (w & kErrOverflow)
        st = -4;
    else if (w & kErrOutOfBox)
        st = -1;
    else if (w & kErrLdsLayout)
        st = -7;
    out[0] = st;
    out[1] = err[1];
}

__global__ void k_split_pairs(const double *__restrict__ acc, int n, double *a, double *b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        if (a)
            a[i] = acc[2 * i];
        if (b)
            b[i] = acc[2 * i + 1];
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers

// Static LDS of the block kernels: the build and the export keep a Hood
// table, the reverse kernel a Hood table and block_sum3's scratch.
static_assert(sizeof(Hood) + 3 * (kMaxThreads / 64) * sizeof(double) <= kBlockStaticLds,
              "static LDS of the block kernels");

hipError_t prepare_kernels(int dyn_bytes) {
    const void *fns[] = {
        reinterpret_cast<const void *>(&k_build<1, kLayoutSoA>),
        reinterpret_cast<const void *>(&k_build<1, kLayoutAoS>),
        reinterpret_cast<const void *>(&k_build<1, kLayoutAoSoA>),
        reinterpret_cast<const void *>(&k_build<2, kLayoutSoA>),
        reinterpret_cast<const void *>(&k_build<2, kLayoutAoS>),
        reinterpret_cast<const void *>(&k_build<2, kLayoutAoSoA>),
        reinterpret_cast<const void *>(&k_force<0, false, 1>),
        reinterpret_cast<const void *>(&k_force<0, true, 1>),
        reinterpret_cast<const void *>(&k_force<1, false, 1>),
        reinterpret_cast<const void *>(&k_force<1, true, 1>),
        reinterpret_cast<const void *>(&k_force<2, false, 1>),
        reinterpret_cast<const void *>(&k_force<2, true, 1>),
        reinterpret_cast<const void *>(&k_force<0, false, 2>),
        reinterpret_cast<const void *>(&k_force<0, true, 2>),
        reinterpret_cast<const void *>(&k_force<1, false, 2>),
        reinterpret_cast<const void *>(&k_force<1, true, 2>),
        reinterpret_cast<const void *>(&k_force<2, false, 2>),
        reinterpret_cast<const void *>(&k_force<2, true, 2>),
        reinterpret_cast<const void *>(&k_force<0, false, 4>),
        reinterpret_cast<const void *>(&k_force<0, true, 4>),
        reinterpret_cast<const void *>(&k_force<1, false, 4>),
        reinterpret_cast<const void *>(&k_force<1, true, 4>),
        reinterpret_cast<const void *>(&k_force<2, false, 4>),
        reinterpret_cast<const void *>(&k_force<2, true, 4>),
        reinterpret_cast<const void *>(&k_force_sd<0, false>),
        reinterpret_cast<const void *>(&k_force_sd<0, true>),
        reinterpret_cast<const void *>(&k_force_sd<1, false>),
        reinterpret_cast<const void *>(&k_force_sd<1, true>),
        reinterpret_cast<const void *>(&k_force_sd<2, false>),
        reinterpret_cast<const void *>(&k_force_sd<2, true>),
        reinterpret_cast<const void *>(&k_force<0, false, 1, true>),
        reinterpret_cast<const void *>(&k_force<0, true, 1, true>),
        reinterpret_cast<const void *>(&k_force<1, false, 1, true>),
        reinterpret_cast<const void *>(&k_force<1, true, 1, true>),
        reinterpret_cast<const void *>(&k_force<2, false, 1, true>),
        reinterpret_cast<const void *>(&k_force<2, true, 1, true>),
        reinterpret_cast<const void *>(&k_hvp<1>),
        reinterpret_cast<const void *>(&k_hvp<2>),
        reinterpret_cast<const void *>(&k_hvp<4>),
    };
    for (const void *f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_bytes);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_gather(const Dims &d, const double *const src[3], const int32_t *orig, const Pos &dst,
                         hipStream_t s) {
    k_gather<<<atom_blocks(d.nt), kAtomThreads, 0, s>>>(d.nt, src ? src[0] : nullptr, src ? src[1] : nullptr,
                                                         src ? src[2] : nullptr, orig, dst);
    return hipGetLastError();
}

// Lanes per atom of the reverse kernel: the most (up to four) whose lanes
// for a workgroup's mean atom count fit one workgroup; threads: those lanes
// for the mean atom count, in whole wavefronts.  Its 48-byte LDS slots often
// leave room for one workgroup per CU only, which more lanes fill with
// wavefronts.
static void hvp_shape(const Dims &d, int &lanes, int &threads) {
    const double per_wg = double(d.nt) / (double(d.nblk) * d.parts);
    lanes = per_wg * 4.0 <= double(kHvpThreads) ? 4 : (per_wg * 2.0 <= double(kHvpThreads) ? 2 : 1);
    threads = std::min(kHvpThreads, std::max(64, round_up(int(per_wg * lanes + 0.5), 64)));
}

hipError_t launch_hvp(const Dims &d, Buffers &b, const Pos &x, const Pos &w, const Pos &lam_x, const Pos &wout,
                      double mult, bool drift_adj, double *partials, hipStream_t s) {
    int L = 1, threads = 64;
    hvp_shape(d, L, threads);
    const size_t lds = 2 * hood_lds_bytes(d.cap);
    const int grid = block_grid(d.nblk * d.parts), da = drift_adj ? 1 : 0;
    if (L == 4)
        k_hvp<4><<<grid, threads, lds, s>>>(d, b.boxes, b.blk_box, x, b.hood_tab, b.nbr_count, b.nbr, w, lam_x, wout,
                                            mult, da, partials);
    else if (L == 2)
        k_hvp<2><<<grid, threads, lds, s>>>(d, b.boxes, b.blk_box, x, b.hood_tab, b.nbr_count, b.nbr, w, lam_x, wout,
                                            mult, da, partials);
    else
        k_hvp<1><<<grid, threads, lds, s>>>(d, b.boxes, b.blk_box, x, b.hood_tab, b.nbr_count, b.nbr, w, lam_x, wout,
                                            mult, da, partials);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const Dims &d, const Buffers &b, const double *partials, double mult, double *acc,
                              hipStream_t s) {
    k_grad_reduce<<<d.nbox, 64, 0, s>>>(b.boxes, partials, d.parts, mult, acc);
    return hipGetLastError();
}

hipError_t launch_traj_sentinels(double *traj, int64_t np, int nt, int count, hipStream_t s) {
    if (count <= 0)
        return hipSuccess;
    k_traj_sentinels<<<(3 * count + 255) / 256, 256, 0, s>>>(traj, np, nt, count);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) {
    if (n <= 0)
        return hipSuccess;
    k_fill_f64<<<int((n + 255) / 256), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_split_pairs(const double *acc, int n, double *a, double *b, hipStream_t s) {
    k_split_pairs<<<(n + 63) / 64, 64, 0, s>>>(acc, n, a, b);
    return hipGetLastError();
}

hipError_t launch_store_box(Box *dst, const Box &B, hipStream_t s) {
    k_store_box<<<1, 64, 0, s>>>(dst, B);
    return hipGetLastError();
}

hipError_t launch_status_out(const int32_t *err, int32_t *out, hipStream_t s) {
    k_status_out<<<1, 64, 0, s>>>(err, out);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0)
        return hipSuccess;
    k_fill_i32<<<int((n + 255) / 256), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_load_state(const Dims &d, const double *const pos[3], const double *const vel[3], Buffers &b,
                             Cursor c, hipStream_t s) {
    const double *v0 = vel ? vel[0] : nullptr, *v1 = vel ? vel[1] : nullptr, *v2 = vel ? vel[2] : nullptr;
    k_load_state<<<atom_blocks(d.nt), kAtomThreads, 0, s>>>(d, b.boxes, b.atom_box, pos[0], pos[1], pos[2], v0,
                                                             v1, v2, pos_layout(d, b.pos(c.x)), b.vx[c.v], b.vy[c.v],
                                                             b.vz[c.v], b.orig[c.o], pos_layout(d, b.pos(1 - c.x)),
                                                             b.err);
    return hipGetLastError();
}

hipError_t launch_unload(const Dims &d, const double *ax, const double *ay, const double *az, const int32_t *orig,
                         double *const out[3], hipStream_t s) {
    k_unload<<<atom_blocks(d.nt), kAtomThreads, 0, s>>>(d.nt, ax, ay, az, orig, out[0], out[1], out[2]);
    return hipGetLastError();
}

hipError_t launch_unload_pos(const Dims &d, const Buffers &b, const Pos &p, const int32_t *orig, double *const out[3],
                             hipStream_t s) {
    k_unload_pos<<<atom_blocks(d.nt), kAtomThreads, 0, s>>>(d.nt, pos_layout(d, p), orig, out[0], out[1], out[2],
                                                             b.boxes, b.atom_box);
    return hipGetLastError();
}

hipError_t launch_relayout(const Dims &d, Buffers &b, Cursor c, int layout, hipStream_t s) {
    Dims to = d;
    to.layout = layout;
    k_relayout<<<(d.ntp + kAtomThreads - 1) / kAtomThreads, kAtomThreads, 0, s>>>(d.ntp, pos_layout(d, b.pos(c.x)),
                                                                                pos_layout(to, b.pos(1 - c.x)));
    // the old buffer's sentinel in the new layout, once the copy has read
    // it (its new place may hold another atom's coordinate in the old one)
    k_put_sentinel<<<1, 1, 0, s>>>(d.nt, pos_layout(to, b.pos(c.x)));
    return hipGetLastError();
}

hipError_t launch_bin(const Dims &d, Buffers &b, Cursor c, bool counts_clear, hipStream_t s) {
    const int xc = c.x, xn = 1 - c.x, o = c.o, on = 1 - c.o, v = c.v, vn = 1 - c.v;
    const int nbin = d.ncs * kSub;
    if (!counts_clear) {
        const hipError_t e = launch_fill_i32(b.cell_count, 0, nbin, s);
        if (e != hipSuccess)
            return e;
    }
    k_bin_count<<<atom_blocks(d.nt), kAtomThreads, 0, s>>>(d, b.boxes, b.atom_box, pos_layout(d, b.pos(xc)),
                                                            b.cell_of, b.slot, b.cell_count, b.err);
    if (nbin <= kScanOne) {
        k_scan_one<<<1, 1024, 0, s>>>(b.cell_count, b.cell_start, nbin);
    } else {
        const int nt = scan_blocks(nbin);
        k_scan_tiles<<<nt, 256, 0, s>>>(b.cell_count, b.cell_start, b.scan_sums, nbin);
        k_scan_add<<<(nbin + 255) / 256, 256, 0, s>>>(b.cell_start, b.scan_sums, nt, nbin);
    }
    k_scatter<<<atom_blocks(d.nt), kAtomThreads, 0, s>>>(d.nt, b.cell_of, b.slot, b.cell_start, b.tmp_idx);
    k_rank_permute<<<atom_blocks(d.nt), kAtomThreads, 0, s>>>(d.nt, d.nbox, b.boxes, b.atom_box, b.tmp_idx, b.cell_of,
                                                               b.cell_start, pos_layout(d, b.pos(xc)), b.vx[v],
                                                               b.vy[v], b.vz[v], b.orig[o], pos_layout(d, b.pos(xn)),
                                                               b.vx[vn], b.vy[vn], b.vz[vn], b.orig[on]);
    return hipGetLastError();
}

hipError_t launch_build(const Dims &d, Buffers &b, Cursor c, hipStream_t s) {
#define TMD_BUILD(BL, LAY)                                                                                          \
    k_build<BL, LAY><<<block_grid(d.nblk * d.parts), d.bthreads, hood_lds_bytes(d.cap), s>>>(                          \
        d, b.boxes, b.blk_box, b.x[c.x], b.cell_start, b.hood_tab, b.nbr_count, b.nbr, b.err)
    switch ((d.blanes == 2 ? 3 : 0) + d.layout) {
    case 0: TMD_BUILD(1, kLayoutSoA); break;
    case 1: TMD_BUILD(1, kLayoutAoS); break;
    case 2: TMD_BUILD(1, kLayoutAoSoA); break;
    case 3: TMD_BUILD(2, kLayoutSoA); break;
    case 4: TMD_BUILD(2, kLayoutAoS); break;
    case 5: TMD_BUILD(2, kLayoutAoSoA); break;
    default: return hipErrorInvalidValue;
    }
#undef TMD_BUILD
    return hipGetLastError();
}

template <int MODE, bool THERMO, int L>
static void force_variant(const Dims &d, Buffers &b, const Pos &in, const Pos &out, int o, hipStream_t s) {
    k_force<MODE, THERMO, L><<<block_grid(d.nblk * d.parts), d.threads, force_lds_bytes(d.cap), s>>>(
        d, b.boxes, b.blk_box, in.x, b.hood_tab, b.nbr_count, b.nbr, b.vx[o], b.vy[o], b.vz[o], b.fx, b.fy, b.fz,
        out.x, b.partials, b.err);
}

template <int MODE, bool THERMO>
static void force_half_variant(const Dims &d, Buffers &b, const Pos &in, const Pos &out, int o, hipStream_t s) {
    k_force<MODE, THERMO, 1, true><<<block_grid(d.nblk * d.parts), d.threads, force_half_lds_bytes(d.cap, d.rcap), s>>>(
        d, b.boxes, b.blk_box, in.x, b.hood_tab, b.nbr_count, b.nbr, b.vx[o], b.vy[o], b.vz[o], b.fx, b.fy, b.fz,
        out.x, b.partials, b.err);
}

template <int MODE, bool THERMO>
static void force_sd_variant(const Dims &d, Buffers &b, const Pos &in, const Pos &out, int o, hipStream_t s) {
    const int vo = MODE >= 1 ? 1 - o : o;  // kicked velocities go to the other half
    k_force_sd<MODE, THERMO><<<block_grid(d.nblk * d.parts), d.threads, 2 * hood_lds_bytes(d.cap), s>>>(
        d, b.boxes, b.blk_box, in, b.hood_tab, b.nbr_count, b.nbr, Pos{b.vx[o], b.vy[o], b.vz[o]},
        Pos{b.vx[vo], b.vy[vo], b.vz[vo]}, Pos{b.fx, b.fy, b.fz}, out, b.partials, b.err);
}

hipError_t launch_force_at(const Dims &d, Buffers &b, const Pos &in, const Pos &out, int o, int mode, bool thermo,
                           hipStream_t s) {
    if (d.model == 1) {  // Spring-Dashpot: one lane per sphere
        switch (mode * 2 + (thermo ? 1 : 0)) {
        case 0: force_sd_variant<0, false>(d, b, in, out, o, s); break;
        case 1: force_sd_variant<0, true>(d, b, in, out, o, s); break;
        case 2: force_sd_variant<1, false>(d, b, in, out, o, s); break;
        case 3: force_sd_variant<1, true>(d, b, in, out, o, s); break;
        case 4: force_sd_variant<2, false>(d, b, in, out, o, s); break;
        case 5: force_sd_variant<2, true>(d, b, in, out, o, s); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (d.half) {  // half lists: one lane per atom
        switch (mode * 2 + (thermo ? 1 : 0)) {
        case 0: force_half_variant<0, false>(d, b, in, out, o, s); break;
        case 1: force_half_variant<0, true>(d, b, in, out, o, s); break;
        case 2: force_half_variant<1, false>(d, b, in, out, o, s); break;
        case 3: force_half_variant<1, true>(d, b, in, out, o, s); break;
        case 4: force_half_variant<2, false>(d, b, in, out, o, s); break;
        case 5: force_half_variant<2, true>(d, b, in, out, o, s); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const int l = d.lpa == 4 ? 2 : (d.lpa == 2 ? 1 : 0);
    switch ((mode * 2 + (thermo ? 1 : 0)) * 3 + l) {
    case 0: force_variant<0, false, 1>(d, b, in, out, o, s); break;
    case 1: force_variant<0, false, 2>(d, b, in, out, o, s); break;
    case 2: force_variant<0, false, 4>(d, b, in, out, o, s); break;
    case 3: force_variant<0, true, 1>(d, b, in, out, o, s); break;
    case 4: force_variant<0, true, 2>(d, b, in, out, o, s); break;
    case 5: force_variant<0, true, 4>(d, b, in, out, o, s); break;
    case 6: force_variant<1, false, 1>(d, b, in, out, o, s); break;
    case 7: force_variant<1, false, 2>(d, b, in, out, o, s); break;
    case 8: force_variant<1, false, 4>(d, b, in, out, o, s); break;
    case 9: force_variant<1, true, 1>(d, b, in, out, o, s); break;
    case 10: force_variant<1, true, 2>(d, b, in, out, o, s); break;
    case 11: force_variant<1, true, 4>(d, b, in, out, o, s); break;
    case 12: force_variant<2, false, 1>(d, b, in, out, o, s); break;
    case 13: force_variant<2, false, 2>(d, b, in, out, o, s); break;
    case 14: force_variant<2, false, 4>(d, b, in, out, o, s); break;
    case 15: force_variant<2, true, 1>(d, b, in, out, o, s); break;
    case 16: force_variant<2, true, 2>(d, b, in, out, o, s); break;
    case 17: force_variant<2, true, 4>(d, b, in, out, o, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_force(const Dims &d, Buffers &b, Cursor c, int mode, bool thermo, hipStream_t s) {
    return launch_force_at(d, b, b.pos(c.x), b.pos(1 - c.x), c.v, mode, thermo, s);
}

hipError_t launch_drift_at(const Dims &d, Buffers &b, const Pos &in, const Pos &out, int o, hipStream_t s) {
    k_drift<<<atom_blocks(d.nt), kAtomThreads, 0, s>>>(d, b.boxes, b.atom_box, in.x, b.vx[o], b.vy[o], b.vz[o], b.fx,
                                                        b.fy, b.fz, out.x, b.err);
    return hipGetLastError();
}

hipError_t launch_drift(const Dims &d, Buffers &b, Cursor c, hipStream_t s) {
    return launch_drift_at(d, b, b.pos(c.x), b.pos(1 - c.x), c.v, s);
}

hipError_t launch_reduce(const Dims &d, const Buffers &b, double *out, int row_len, hipStream_t s) {
    k_reduce<<<d.nbox, 64, 0, s>>>(b.boxes, b.partials, d.parts, out, row_len);
    return hipGetLastError();
}

hipError_t launch_export_neighbors(const Dims &d, const Buffers &b, Cursor c, int32_t *counts, int32_t *ids,
                                   hipStream_t s) {
    k_export_neighbors<<<block_grid(d.nblk), d.bthreads, 0, s>>>(d, b.boxes, b.blk_box, b.cell_start, b.nbr_count,
                                                                b.nbr, b.orig[c.o], counts, ids);
    return hipGetLastError();
}

}  // namespace tmd

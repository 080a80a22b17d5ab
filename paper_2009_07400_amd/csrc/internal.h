// Internal declarations shared by the C-ABI layer (api.hip) and the kernels
// (engine.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmd {

constexpr int kScanTile = 1024;    // elements per workgroup in the cell-count scan
constexpr int kScanOne = 32768;    // bin slots up to which one workgroup scans (and clears) the counts
constexpr int kPartialStride = 4;  // doubles per block partial: U, W, KE, pad
constexpr int kNumXcd = 8;         // MI355X: 8 accelerator complex dies, each with its own L2
constexpr int kMaxEdge = 3;        // cells per block edge: 2 or 3 (a whole small box: up to kWholeBoxCells)
constexpr int kWholeBoxCells = 4;  // boxes of at most this many (and E + 2) cells per axis are one block
constexpr int kMaxHood = 125;      // cells in a block neighborhood (at most edge + 2 per axis)
constexpr int kMaxThreads = 1024;  // threads per block workgroup (upper bound)
constexpr int kAtomThreads = 256;  // threads per workgroup of per-atom kernels
constexpr int kMaxParts = 4;       // workgroups per block, at most
constexpr int kHoodWords = 256;    // int32 words of one block's stored neighborhood table
// Binning sorts atoms by cell and, inside a cell, by subcell: the cell cut
// in 2 x 2 x 2 (subcell index (sz * 2 + sy) * 2 + sx), then by original id.
// Bin slot of subcell k of cell slot c: c * kSub + k.
constexpr int kSub = 8;
constexpr int kMaxSubGrid = kSub * kMaxHood;  // subcells of a block neighborhood, at most

// Bits of the device error word err[0].
constexpr int kErrOverflow = 1;
constexpr int kErrNonFinite = 2;
constexpr int kErrOutOfBox = 4;  // set_state got a coordinate outside [-L, 2L)
constexpr int kErrLdsLayout = 8; // the force kernel's dynamic LDS does not start at address 0

// One periodic cubic box.  Cells are numbered block-major: a block is E x E x
// E cells (E = 2 or 3; thinner at the high faces when E does not divide the
// cell count; a box of at most min(E + 2, kWholeBoxCells) cells per axis is
// one block of all its cells), each block owns edge^3 consecutive cell
// slots, so the atoms of a block and of each of its cells are contiguous
// after binning.
struct Box {
    int32_t atom_off, n;     // atoms [atom_off, atom_off + n) of the concatenated arrays
    int32_t cell_off, nc;    // first cell slot; cells per axis
    int32_t nbx, block_off;  // blocks per axis (ceil(nc / E)); first block
    int32_t nblocks, edge;   // blocks of this box; its block edge: E, or nc when the box is one block
    double L, halfL, side;   // box, half box, cell side L / nc
    double hside;            // subcell side: side / 2
    double halfL2;           // (L/2)^2
    double invL;             // 1 / L
    double rc2, rl2;         // cutoff^2, (cutoff + skin)^2
    double eps, sigma6;      // LJ parameters
    double eps48, eps24;     // 48 eps and 24 eps: f = sr2 sr6 (48 eps sr6 - 24 eps)
    double eps4;             // 4 eps: pair energy sr6 (4 eps sr6 - 4 eps)
    double eps_over_sigma;   // d f / d sigma = (eps / sigma) sr2 sr6 (576 sr6 - 144)
    double f12, f6;          // 48 eps sigma^12, 24 eps sigma^6: f = sr2 q (f12 q - f6) with q = sr2^3
    double u12, u6;          // 4 eps sigma^12, 4 eps sigma^6: pair energy q (u12 q - u6)
    // derivative constants (q = sr2^3): df/ds = sr2^2 q (4 f6 - 7 f12 q), so
    // 2 df/ds = sr2^2 q (g8 - g14 q); df/deps = sr2 q (e12 q - e6);
    // df/dsigma = sr2 q (h12 q - h6)
    double g14, g8;          // 14 f12, 8 f6
    double e12, e6;          // f12 / eps, f6 / eps
    double h12, h6;          // 12 f12 / sigma, 6 f6 / sigma
    double h, dt, mass;      // half kick dt / (2 m), time step, mass
    // Spring-Dashpot contact (model 1): spring constant K, dissipation
    // gamma, diameter sigma and sigma^2
    double sd_k, sd_g, sd_sig, sd_sig2;
};

// Sizes shared by all kernels of one system.
struct Dims {
    int32_t nt;       // atoms in all boxes
    int32_t ntp;      // padded stride of the neighbor-major list
    int32_t nbox;     // boxes
    int32_t nblk;     // blocks in all boxes
    int32_t ncs;      // cell slots in all boxes (Box.edge^3 per block); kSub bin slots each
    int32_t edge;     // E, cells per block edge
    int32_t maxnb;    // list capacity per atom
    int32_t cap;      // atoms a block neighborhood may stage in LDS
    int32_t threads;  // threads per force workgroup (64..kMaxThreads, multiple of 64)
    int32_t bthreads; // threads per workgroup of the one-lane-per-atom block kernels (list build, adjoint, export)
    int32_t nchunk;   // 4-entry list chunks per atom: ceil(maxnb / 4) + 1 (a spare chunk of padding)
    int32_t parts;    // workgroups per block (1, 2 or 4), each taking a share of the block's atoms
    int32_t lpa;      // lanes per atom in the force kernel (1, 2 or 4), each taking every lpa-th list chunk
    int32_t blanes;   // lanes per atom in the list build (1 or 2)
    int32_t model;    // force model of every box: 0 Lennard-Jones, 1 Spring-Dashpot
    int32_t half;     // 1: half lists inside blocks (Newton's third law in the force kernel's LDS)
    int32_t rcap;     // LDS slots of a block's reaction sums with half lists (0 without)
    int32_t layout;   // position layout: 0 SoA, 1 AoS, 2 AoSoA of 64-atom clusters (PosL)
};

// Neighbor list layout: neighbor-major within tiles of 64 atoms (one
// wavefront) and chunks of 4 entries.  Entry k of atom i lives at
//   ((tile(i) * nchunk + k / 4) * 64 + lane(i)) * 4 + k % 4,
// so one 16-byte load gives a lane four consecutive entries, a wavefront's
// chunk is one contiguous 1 KB row, and a tile's whole list is one
// contiguous stretch of nchunk KB that a wavefront streams through in order.
__host__ __device__ inline int64_t nbr_index(int i, int k, int nchunk) {
    return ((int64_t((i >> 6)) * nchunk + (k >> 2)) * 64 + (i & 63)) * 4 + (k & 3);
}

// Atoms of blocks whose neighborhood is staged in LDS store 16-bit LDS slots
// instead, eight to a 16-byte chunk, in the same rows: entry k of atom i is
// uint16 element
//   ((tile(i) * nchunk + k / 8) * 64 + lane(i)) * 8 + k % 8.
__host__ __device__ inline int64_t nbr_index16(int i, int k, int nchunk) {
    return ((int64_t((i >> 6)) * nchunk + (k >> 3)) * 64 + (i & 63)) * 8 + (k & 7);
}

// Three SoA coordinate arrays.
struct Pos {
    double *x, *y, *z;
};

// One position buffer of 3 ntp doubles in one of the particle layouts of
// Sec. 4.2 (ArrayLayout): 0 SoA (column-major: x of every atom, then y,
// then z), 1 AoS (row-major: x, y, z of an atom side by side), 2 AoSoA
// (clustered: 64 atoms - one wavefront - per cluster, their 64 x, 64 y and
// 64 z in turn).  Every layout keeps slot nt (the NaN sentinel atom) and the
// padding below ntp inside the buffer (ntp is a multiple of 256).  Offsets
// are 32-bit (3 ntp < 2^31): the list build keeps fewer registers, and AoS
// and AoSoA reach y and z at constant offsets from x.
enum { kLayoutSoA = 0, kLayoutAoS = 1, kLayoutAoSoA = 2 };

struct PosL {
    double *p;
    int32_t ntp, layout;
    __device__ __forceinline__ void get(int i, double &a, double &b, double &c) const {
        if (layout == kLayoutSoA) {
            a = p[i];
            b = p[i + ntp];
            c = p[i + 2 * ntp];
        } else if (layout == kLayoutAoS) {
            const double *q = p + 3 * i;
            a = q[0];
            b = q[1];
            c = q[2];
        } else {
            const double *q = p + ((i >> 6) * 192 + (i & 63));
            a = q[0];
            b = q[64];
            c = q[128];
        }
    }
    __device__ __forceinline__ void put(int i, double a, double b, double c) const {
        if (layout == kLayoutSoA) {
            p[i] = a;
            p[i + ntp] = b;
            p[i + 2 * ntp] = c;
        } else if (layout == kLayoutAoS) {
            double *q = p + 3 * i;
            q[0] = a;
            q[1] = b;
            q[2] = c;
        } else {
            double *q = p + ((i >> 6) * 192 + (i & 63));
            q[0] = a;
            q[64] = b;
            q[128] = c;
        }
    }
};

// The buffer behind a Pos whose y and z follow x at strides of ntp (every
// position buffer of the workspace and of the adjoint's storage), read in
// layout d.layout.
inline PosL pos_layout(const Dims &d, const Pos &q) { return PosL{q.x, d.ntp, d.layout}; }

// Device pointers carved from the caller's workspace.
struct Buffers {
    Pos pos(int k) const { return Pos{x[k], y[k], z[k]}; }
    double *x[2], *y[2], *z[2];
    double *vx[2], *vy[2], *vz[2];
    int32_t *orig[2];
    double *fx, *fy, *fz;
    Box *boxes;            // [nbox]  (uploaded at set_state)
    int32_t *blk_box;      // [nblk]  box of each block
    int32_t *atom_box;     // [nt]    box of each atom slot (boxes keep fixed slot ranges)
    int32_t *cell_of, *slot, *tmp_idx;
    int32_t *cell_count, *cell_start, *scan_sums;  // per bin slot (kSub per cell slot)
    int32_t *nbr_count, *nbr;
    int32_t *hood_tab;     // [nblk][kHoodWords] neighborhood tables, written by every list build
    double *partials;      // [nblk * parts][kPartialStride]
    int32_t *err;          // [0] flags, [1] largest list length requested on overflow
};

// Which half of each double buffer is current: positions flip on every drift
// and every binning; original ids flip only on binning.  Velocities flip on
// binning, and for the Spring-Dashpot model also at every force launch that
// kicks them: its force reads neighbours' velocities, so the kicked ones go
// to the other half (Lennard-Jones kicks them in place).
struct Cursor {
    int x = 0;
    int o = 0;
    int v = 0;
};

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }
inline int atom_blocks(int n) { return (n + kAtomThreads - 1) / kAtomThreads; }
inline int scan_blocks(int ncell) { return (ncell + kScanTile - 1) / kScanTile; }
// Grid of block workgroups: a multiple of the XCD count so the remap in the
// kernels gives every XCD one contiguous range of blocks.
inline int block_grid(int nblk) { return round_up(nblk, kNumXcd); }
// LDS bytes of a block workgroup staging `cap` atoms plus the NaN sentinel
// and one scratch slot.
// LDS slots past a neighborhood copy's capacity: the NaN sentinel (slot cap),
// a scratch slot for the staging's unconditional writes (cap + 1), and
// kHoodPad slots that the two-lane list build may read past a run's end
// (unused values, masked out) so that its candidate reads need no clamping.
constexpr int kHoodPad = 8;
inline size_t hood_lds_bytes(int cap) { return size_t(cap + 2 + kHoodPad) * 3 * sizeof(double); }

// The force kernel keeps no static LDS: its dynamic LDS holds the
// neighborhood copy from address 0, then its neighborhood table and
// reduction scratch in kForceLdsTail bytes.
constexpr int kForceLdsTail = 1536;
inline size_t force_lds_bytes(int cap) { return hood_lds_bytes(cap) + kForceLdsTail; }

// Half lists: a block's reaction sums cover the LDS slots from its first
// own cell's to its last own cell's (22 of the 64 neighborhood cells at edge
// 2, 63 of 125 at edge 3), rcap slots of 24 bytes after the force kernel's
// tail; blocks whose span is larger keep full lists.
inline size_t force_half_lds_bytes(int cap, int rcap) {
    return force_lds_bytes(cap) + size_t(rcap) * 3 * sizeof(double);
}

// Upper bound of the static LDS any block kernel declares (neighborhood
// table, reduction scratch); engine.hip checks its kernels against it.
constexpr int kBlockStaticLds = 1536;

// Launchers (engine.hip).  All enqueue on `s` and return the launch status.
// Allow every block kernel up to dyn_bytes of dynamic LDS on the current
// device (the device's per-workgroup limit less kBlockStaticLds).
hipError_t prepare_kernels(int dyn_bytes);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
// Write one box descriptor (passed by value) to dst.
hipError_t launch_store_box(Box *dst, const Box &B, hipStream_t s);
// out[0] = the status code tmd_sync() would return for the error word err
// (0 when clear), out[1] = largest list length requested on overflow.
hipError_t launch_status_out(const int32_t *err, int32_t *out, hipStream_t s);
// vel == nullptr loads zero velocities.
hipError_t launch_load_state(const Dims &d, const double *const pos[3], const double *const vel[3], Buffers &b,
                             Cursor c, hipStream_t s);
hipError_t launch_unload(const Dims &d, const double *ax, const double *ay, const double *az, const int32_t *orig,
                         double *const out[3], hipStream_t s);
// launch_unload for positions, wrapped into [0, L) on the way.
hipError_t launch_unload_pos(const Dims &d, const Buffers &b, const Pos &p, const int32_t *orig, double *const out[3],
                             hipStream_t s);
// Copy the current positions (half c.x, layout d.layout) into the other half
// in `layout`, with the NaN sentinel in both halves in that layout; the
// caller then flips c.x.
hipError_t launch_relayout(const Dims &d, Buffers &b, Cursor c, int layout, hipStream_t s);
// Binning (both halves flip).  counts_clear: the cell counts are known to be
// zero (left so by the previous binning's one-workgroup scan), which skips
// clearing them first.
hipError_t launch_bin(const Dims &d, Buffers &b, Cursor c, bool counts_clear, hipStream_t s);
hipError_t launch_build(const Dims &d, Buffers &b, Cursor c, hipStream_t s);
// mode 0: F only (stored); 1: F + kick (stored, end of integrate);
// 2: F + kick + kick + drift into positions 1 - c.x.  Velocities are read
// from half c.v; the Spring-Dashpot model writes kicked ones to half 1 - c.v
// (the caller then flips c.v), Lennard-Jones in place.
hipError_t launch_force(const Dims &d, Buffers &b, Cursor c, int mode, bool thermo, hipStream_t s);
hipError_t launch_drift(const Dims &d, Buffers &b, Cursor c, hipStream_t s);  // positions into 1 - c.x
// The same with explicit position arrays (in: current, out: drifted) and
// velocity half o (kicked velocities as in launch_force); used to recompute
// a trajectory segment into storage and to time the kernel.
hipError_t launch_force_at(const Dims &d, Buffers &b, const Pos &in, const Pos &out, int o, int mode, bool thermo,
                           hipStream_t s);
hipError_t launch_drift_at(const Dims &d, Buffers &b, const Pos &in, const Pos &out, int o, hipStream_t s);

// Adjoint support.
// Gather a vector field from original order into the current sorted order
// (dst[p] = src[orig[p]]) or scatter it back (launch_unload does that).
hipError_t launch_gather(const Dims &d, const double *const src[3], const int32_t *orig, const Pos &dst,
                         hipStream_t s);
// One reverse step at force point x: lam_x += c J(x) w with c = mult * h
// (per box), w = lam_v; per-block partials of w . dF/deps and w . dF/dsigma;
// with drift_adj, wout = w + dt lam_x (the adjoint of the preceding drift).
hipError_t launch_hvp(const Dims &d, Buffers &b, const Pos &x, const Pos &w, const Pos &lam_x, const Pos &wout,
                      double mult, bool drift_adj, double *partials, hipStream_t s);
// acc[2 box + {0, 1}] += mult * h_box * (sum of the box's partials), in a fixed order.
hipError_t launch_grad_reduce(const Dims &d, const Buffers &b, const double *partials, double mult, double *acc,
                              hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
// NaN sentinel atom (slot nt) in position buffers 1..count of a trajectory
// store laid out as [count + 1][3][np].
hipError_t launch_traj_sentinels(double *traj, int64_t np, int nt, int count, hipStream_t s);
// a[i] = acc[2 i], b[i] = acc[2 i + 1] for i < n (either output nullable).
hipError_t launch_split_pairs(const double *acc, int n, double *a, double *b, hipStream_t s);
// Per-box deterministic sums of the block partials: rows of (U, W) when
// row_len == 2, (KE, T, U, W, E) when row_len == 5; out holds nbox rows.
hipError_t launch_reduce(const Dims &d, const Buffers &b, double *out, int row_len, hipStream_t s);
hipError_t launch_export_neighbors(const Dims &d, const Buffers &b, Cursor c, int32_t *counts, int32_t *ids,
                                   hipStream_t s);

}  // namespace tmd

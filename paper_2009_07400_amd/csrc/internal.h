// Internal declarations shared by the C-ABI layer (api.hip) and the kernels.
// Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmd {

constexpr int kBlock = 256;      // threads per workgroup for per-atom kernels (4 wave64)
constexpr int kScanTile = 1024;  // elements per workgroup in the cell-count scan
constexpr int kPartialStride = 4;  // doubles per workgroup partial: U, W, KE, pad
constexpr int kNumXcd = 8;       // MI355X: 8 accelerator complex dies, each with its own L2

// Bits of the device error word err[0].
constexpr int kErrOverflow = 1;
constexpr int kErrNonFinite = 2;
constexpr int kErrOutOfBox = 4;  // set_state got a coordinate outside [-L, 2L)

// Everything a kernel needs to know about one periodic box.
struct Geom {
    int32_t n;       // atoms
    int32_t np;      // padded stride of per-atom arrays and neighbor-major rows
    int32_t nc;      // cells per axis
    int32_t ncell;   // nc^3
    int32_t maxnb;   // list capacity per atom
    int32_t pad_;
    double L, halfL, side;  // box, half box, cell side L / nc
    double rc2, rl2;        // cutoff^2, (cutoff + skin)^2
    double eps, sigma6;     // LJ parameters
    double h, dt;           // half kick dt / (2 m), time step
    double mass;
};

// Device pointers carved from the caller's workspace.  Positions, velocities
// and original ids are double-buffered: binning permutes buffer `cur` into
// the other one, and the fused force/drift kernel writes new positions there.
struct Buffers {
    double *x[2], *y[2], *z[2];
    double *vx[2], *vy[2], *vz[2];
    int32_t *orig[2];
    double *fx, *fy, *fz;
    int32_t *cell_of, *slot, *tmp_idx;
    int32_t *cell_count, *cell_start, *scan_sums;
    int32_t *nbr_count, *nbr;
    double *partials;
    double *scalars;  // small scratch for reductions
    int32_t *err;     // [0] flags, [1] largest list length requested on overflow
};

// Grid size for per-atom kernels: a multiple of the XCD count so the
// blockIdx remap below gives every XCD one contiguous range of atoms.
inline int atom_grid(int n) {
    int g = (n + kBlock - 1) / kBlock;
    return ((g + kNumXcd - 1) / kNumXcd) * kNumXcd;
}
inline int scan_blocks(int ncell) { return (ncell + kScanTile - 1) / kScanTile; }

// Which half of each double buffer is current: positions flip on every drift
// and every binning; velocities and original ids flip only on binning (the
// kicks update velocities in place).
struct Cursor {
    int x = 0;  // positions
    int o = 0;  // atom order: velocities and original ids
};

// Launchers (kernels.hip).  All enqueue on `s` and return the launch status.
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_load_state(const Geom &g, const double *const pos[3], const double *const vel[3],
                             Buffers &b, Cursor c, hipStream_t s);
hipError_t launch_unload(const Geom &g, const double *ax, const double *ay, const double *az,
                         const int32_t *orig, double *const out[3], hipStream_t s);
hipError_t launch_bin(const Geom &g, Buffers &b, Cursor c, hipStream_t s);  // both halves flip
hipError_t launch_build(const Geom &g, Buffers &b, Cursor c, hipStream_t s);
// mode 0: F only (stored); 1: F + kick (stored, end of integrate); 2: F + kick + kick + drift into 1 - c.x
hipError_t launch_force(const Geom &g, Buffers &b, Cursor c, int mode, bool thermo, hipStream_t s);
hipError_t launch_drift(const Geom &g, Buffers &b, Cursor c, hipStream_t s);  // positions into 1 - c.x
// Deterministic sum of the force kernel's workgroup partials.  Writes
// (U, W) when row_len == 2 or (KE, T, U, W, E) when row_len == 5.
hipError_t launch_reduce(const Geom &g, const Buffers &b, double *out, int row_len, hipStream_t s);
hipError_t launch_export_neighbors(const Geom &g, const Buffers &b, Cursor c, int32_t *counts, int32_t *ids,
                                   hipStream_t s);

}  // namespace tmd

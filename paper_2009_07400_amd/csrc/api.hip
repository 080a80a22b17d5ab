// C-ABI layer of the MI355X Lennard-Jones MD library: argument checking,
// box and block tables, workspace carving, call ordering, the integration
// schedule, kernel tuning and deferred device errors.  Every numerical step
// runs in the kernels of engine.hip.
#include "tmd.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace tmd;

struct tmd_system {
    std::vector<Box> boxes;  // host copy of the descriptors
    std::vector<int32_t> blk_box, atom_box;
    Dims d{};
    Dims dmax{};               // sizes the workspace for either block edge
    bool tables_dirty = true;  // box / block tables changed since the last upload
    bool counts_clear = false; // cell counts left at zero by the last binning
    int32_t rebuild_every = 20;
    size_t ws_need = 0;
    Buffers b{};
    Cursor cur;
    bool bound = false, have_state = false, list_valid = false, force_valid = false, prepared = false;
    int64_t step = 0;
    std::string err;
    uint64_t gen = 0;  // bumped by every call that changes the state or the parameters

    // recorded forward run for the adjoint
    struct Adj {
        bool recorded = false;
        int64_t step0 = 0;
        int32_t nsteps = 0, nseg = 0;
        void *ws = nullptr;
        uint64_t gen = 0;
    } adj;

    struct Ev {
        int cls;
        hipEvent_t a, b;
        int n;  // launches between the two events
    };
    bool timing = false;
    std::vector<Ev> pending;
    std::vector<hipEvent_t> pool;
    double t_ms[TMD_T_COUNT] = {};
    int64_t t_n[TMD_T_COUNT] = {};

    // Rebuild intervals of tmd_integrate captured as HIP graphs
    // (tmd_set_graphs).  A graph bakes in the launch parameters, the buffer
    // pointers and which copy of the double-buffered state each launch reads,
    // so it is keyed by all of them; an interval flips the copies, so runs
    // alternate between two graphs.
    struct Seg {
        std::vector<unsigned char> key;
        hipGraphExec_t exec = nullptr;
        Cursor cur_after;
        bool counts_clear_after = false;
    };
    bool graphs = false;
    hipStream_t cap_stream = nullptr;  // capture only: the graphs run on the caller's stream
    std::vector<Seg> segs;
    int32_t graph_captures = 0;
    int64_t graph_launches = 0;
};

namespace {

constexpr size_t kAlign = 256;
// Atoms of a system, at most: the position layouts address a buffer of 3 ntp
// doubles with 32-bit offsets.
constexpr int64_t kMaxAtoms = 700000000;
constexpr int kMaxCap = 4096;       // atoms staged per block neighborhood (96 KB of LDS at most)
constexpr int kLdsPerCu = 163840;   // gfx950: 160 KB of LDS per compute unit
constexpr int kStaticLds = kBlockStaticLds;  // static LDS of a block kernel (neighborhood tables, reductions)
static_assert(kForceLdsTail <= kStaticLds, "the force kernel's table and scratch fit the static LDS allowance");

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Carve the workspace; with base == nullptr only the size is computed.
size_t carve(const Dims &d, char *base, Buffers *out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    const size_t np = size_t(d.ntp);
    Buffers b{};
    for (int k = 0; k < 2; ++k) {
        b.x[k] = (double *)take(np * 8);
        b.y[k] = (double *)take(np * 8);
        b.z[k] = (double *)take(np * 8);
        b.vx[k] = (double *)take(np * 8);
        b.vy[k] = (double *)take(np * 8);
        b.vz[k] = (double *)take(np * 8);
        b.orig[k] = (int32_t *)take(np * 4);
    }
    b.fx = (double *)take(np * 8);
    b.fy = (double *)take(np * 8);
    b.fz = (double *)take(np * 8);
    b.boxes = (Box *)take(size_t(d.nbox) * sizeof(Box));
    b.blk_box = (int32_t *)take(size_t(d.nblk) * 4);
    b.atom_box = (int32_t *)take(np * 4);
    b.cell_of = (int32_t *)take(np * 4);
    b.slot = (int32_t *)take(np * 4);
    b.tmp_idx = (int32_t *)take(np * 4);
    const size_t nbin = size_t(d.ncs) * kSub;
    b.cell_count = (int32_t *)take(nbin * 4);
    b.cell_start = (int32_t *)take((nbin + 1) * 4);
    b.scan_sums = (int32_t *)take((size_t(scan_blocks(int(nbin))) + 1) * 4);
    b.nbr_count = (int32_t *)take(np * 4);
    b.nbr = (int32_t *)take(np * size_t(d.nchunk) * 4 * 4);
    b.hood_tab = (int32_t *)take(size_t(d.nblk) * kHoodWords * 4);
    b.partials = (double *)take(size_t(d.nblk) * kMaxParts * kPartialStride * 8);
    b.err = (int32_t *)take(64);
    if (out)
        *out = b;
    return off;
}

bool positive(double v) { return isfinite(v) && v > 0.0; }

tmd_status fail(tmd_system *s, tmd_status st, const std::string &msg) {
    if (s)
        s->err = msg;
    return st;
}

tmd_status hip_fail(tmd_system *s, hipError_t e, const char *where) {
    return fail(s, TMD_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

hipEvent_t get_event(tmd_system *s) {
    if (!s->pool.empty()) {
        hipEvent_t e = s->pool.back();
        s->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Brackets the kernels of one class with events on the launch stream.
struct Timed {
    tmd_system *s;
    int cls;
    hipStream_t st;
    hipEvent_t a = nullptr;
    Timed(tmd_system *s_, int cls_, hipStream_t st_) : s(s_), cls(cls_), st(st_) {
        if (s->timing && (a = get_event(s)) != nullptr)
            (void)hipEventRecord(a, st);
    }
    ~Timed() {
        if (!a)
            return;
        hipEvent_t b = get_event(s);
        if (!b) {
            s->pool.push_back(a);
            return;
        }
        (void)hipEventRecord(b, st);
        s->pending.push_back({cls, a, b, 1});
    }
};

// Brackets a run of back-to-back launches of one class with one pair of
// events (so the average includes no event overhead between them): add()
// before each launch, close() before a launch of another class.
struct TimedRun {
    tmd_system *s;
    int cls;
    hipStream_t st;
    hipEvent_t a = nullptr;
    int n = 0;
    TimedRun(tmd_system *s_, int cls_, hipStream_t st_) : s(s_), cls(cls_), st(st_) {}
    void add() {
        if (!s->timing)
            return;
        if (n == 0) {
            if ((a = get_event(s)) == nullptr)
                return;
            (void)hipEventRecord(a, st);
        }
        ++n;
    }
    void close() {
        if (n == 0 || !a)
            return;
        hipEvent_t b = get_event(s);
        if (b) {
            (void)hipEventRecord(b, st);
            s->pending.push_back({cls, a, b, n});
        } else {
            s->pool.push_back(a);
        }
        a = nullptr;
        n = 0;
    }
    ~TimedRun() { close(); }
};

tmd_status check_ready(tmd_system *s, bool need_state) {
    if (!s)
        return TMD_EINVAL;
    if (!s->bound)
        return fail(s, TMD_ESTATE, "no workspace bound");
    if (need_state && !s->have_state)
        return fail(s, TMD_ESTATE, "no state set");
    return TMD_OK;
}

tmd_status upload_tables(tmd_system *s, hipStream_t hs);

tmd_status rebuild(tmd_system *s, hipStream_t st) {
    if (s->tables_dirty || !s->prepared) {
        const tmd_status u = upload_tables(s, st);
        if (u != TMD_OK)
            return u;
    }
    hipError_t e;
    {
        Timed t(s, TMD_T_BINNING, st);
        e = launch_bin(s->d, s->b, s->cur, s->counts_clear, st);
        s->counts_clear = e == hipSuccess;  // either scan clears the counts
    }
    if (e != hipSuccess)
        return hip_fail(s, e, "binning");
    s->cur.x = 1 - s->cur.x;
    s->cur.o = 1 - s->cur.o;
    s->cur.v = 1 - s->cur.v;
    {
        Timed t(s, TMD_T_NEIGHBOR, st);
        e = launch_build(s->d, s->b, s->cur, st);
    }
    if (e != hipSuccess)
        return hip_fail(s, e, "neighbor build");
    s->list_valid = true;
    s->force_valid = false;
    s->gen++;
    return TMD_OK;
}

// Threads per block workgroup: the mean number of atoms one workgroup takes
// (a block's atoms split over d.parts workgroups) times the lanes each atom
// gets, rounded up to whole wavefronts.  (More threads than that leave waves
// idle in most blocks and, at two workgroups per CU, unevenly spread over
// the SIMDs; the few fuller blocks take a second pass.)
int default_threads(const Dims &d, int lanes) {
    const double per_wg = double(d.nt) / (double(d.nblk) * d.parts) * lanes;
    return std::min(kMaxThreads, std::max(64, round_up(int(per_wg + 0.5), 64)));
}

// LJ 12-6 constants of one box (Sec. 3.2, Eq. 2) in the forms the kernels use.
void set_lj(Box &B, double eps, double sigma) {
    const double s2 = sigma * sigma;
    B.eps = eps;
    B.sigma6 = s2 * s2 * s2;
    B.eps48 = 48.0 * eps;
    B.eps24 = 24.0 * eps;
    B.eps4 = 4.0 * eps;
    B.eps_over_sigma = eps / sigma;
    B.f12 = B.eps48 * B.sigma6 * B.sigma6;
    B.f6 = B.eps24 * B.sigma6;
    B.u12 = B.eps4 * B.sigma6 * B.sigma6;
    B.u6 = B.eps4 * B.sigma6;
    B.g14 = 14.0 * B.f12;
    B.g8 = 8.0 * B.f6;
    B.e12 = 48.0 * B.sigma6 * B.sigma6;
    B.e6 = 24.0 * B.sigma6;
    B.h12 = 12.0 * B.f12 / sigma;
    B.h6 = 6.0 * B.f6 / sigma;
}

// Expected atoms in a block neighborhood (E + 2 cells per axis, or the whole
// box when it has fewer cells), for sizing the LDS staging area.
double expected_hood_atoms(const Box &B, int E) {
    const double f = double(std::min(B.nc, E + 2)) / B.nc;
    return B.n * f * f * f;
}

// Cut every box into blocks of E x E x E cells and size the schedule for
// it: the LDS capacity is the largest per-workgroup share of a CU's LDS that
// still holds at least 15% more atoms than the largest mean neighborhood
// population (liquid density fluctuations over ~1000 atoms are a few
// percent; rarer blocks fall back to global gathers), threads the mean block
// population rounded up to whole wavefronts.  Fills the block fields of the
// `nbox` descriptors and the Dims fields that follow from them.  Returns
// false when the cell slots overflow int32.
bool layout_dims(Box *boxes, int32_t nbox, int E, Dims &d) {
    int64_t blocks = 0, cells = 0;
    double worst = 0.0;
    for (int32_t k = 0; k < nbox; ++k) {
        Box &B = boxes[k];
        // a box of at most E + 2 (and at most 4) cells per axis is one block:
        // every block's neighborhood would hold the whole box anyway, so one
        // workgroup stages it once instead of each of its blocks staging it
        const int Eb = B.nc <= std::min(E + 2, kWholeBoxCells) ? B.nc : E;
        B.edge = Eb;
        B.nbx = (B.nc + Eb - 1) / Eb;
        B.nblocks = B.nbx * B.nbx * B.nbx;
        B.block_off = int32_t(blocks);
        B.cell_off = int32_t(cells);
        blocks += B.nblocks;
        cells += int64_t(B.nblocks) * Eb * Eb * Eb;
        worst = std::max(worst, expected_hood_atoms(B, Eb));
        if (cells * kSub > INT32_MAX / 2)
            return false;
    }
    d.edge = E;
    d.nblk = int32_t(blocks);
    d.ncs = int32_t(cells);
    // Most workgroups per CU (gfx950: 160 KB of LDS per CU) whose share of
    // LDS still stages at least 15% more atoms than the largest mean
    // neighborhood; the capacity then takes that whole share.
    const int need = int(1.15 * worst) + 32;
    // the Spring-Dashpot force kernel stages velocities too: 48 bytes a slot
    const int slot = d.model == 1 ? 48 : 24;
    // half lists add the reaction sums over the own cells' slot span, sized
    // like the staging area for the same share of the neighborhood's cells
    const double span_cells = E == 2 ? 22.0 / 64.0 : 63.0 / 125.0;
    d.rcap = d.half ? round_up(int(1.15 * worst * span_cells) + 32, 64) : 0;
    d.cap = std::min(kMaxCap, round_up(int(1.3 * worst) + 64, 64));
    for (int wg = 8; wg >= 1; --wg) {
        // + slots past the capacity
        const int c = ((kLdsPerCu / wg - kStaticLds) / slot - 2 - kHoodPad - d.rcap) / 64 * 64;
        if (c >= need) {
            d.cap = std::min(kMaxCap, c);
            break;
        }
    }
    d.rcap = std::min(d.rcap, d.cap);
    if (d.parts < 1)
        d.parts = 1;
    if (d.lpa < 1)
        d.lpa = 1;
    if (d.blanes < 1)
        d.blanes = 1;
    d.threads = default_threads(d, d.lpa);
    d.bthreads = default_threads(d, d.blanes);
    return true;
}

bool layout_blocks(tmd_system *s, int E) {
    Dims &d = s->d;
    if (!layout_dims(s->boxes.data(), d.nbox, E, d))
        return false;
    s->blk_box.assign(size_t(d.nblk), 0);
    for (int32_t k = 0; k < d.nbox; ++k) {
        const Box &B = s->boxes[size_t(k)];
        std::fill(s->blk_box.begin() + B.block_off, s->blk_box.begin() + B.block_off + B.nblocks, k);
    }
    s->tables_dirty = true;
    s->prepared = false;
    s->counts_clear = false;
    return true;
}

// Default block edge: 3 when that still gives every CU several blocks.
int default_edge(const Box *boxes, int32_t nbox) {
    int64_t b3 = 0;
    for (int32_t k = 0; k < nbox; ++k) {
        const int64_t n = (boxes[k].nc + 2) / 3;
        b3 += n * n * n;
    }
    return b3 >= 4 * 256 ? 3 : 2;
}

// Check one box's parameters (the argument rules of tmd_create) and fill
// its descriptor; its atoms start at slot atom_off of the concatenated arrays.
tmd_status make_box(const tmd_params &p, int64_t n, double L, int64_t atom_off, Box &B) {
    if (n <= 0 || n > kMaxAtoms)
        return TMD_EINVAL;
    if (!positive(p.epsilon) || !positive(p.sigma) || !positive(p.mass) || !positive(p.cutoff) ||
        !positive(p.dt) || !positive(L) || !isfinite(p.skin) || p.skin < 0.0)
        return TMD_EINVAL;
    if (p.rebuild_every < 1 || p.max_neighbors < 1 || p.max_neighbors > 4096)
        return TMD_EINVAL;
    if (p.model != TMD_MODEL_LJ && p.model != TMD_MODEL_SPRING_DASHPOT)
        return TMD_EINVAL;
    if (p.model == TMD_MODEL_SPRING_DASHPOT &&
        (!isfinite(p.stiffness) || p.stiffness < 0.0 || !isfinite(p.damping) || p.damping < 0.0 ||
         !(p.cutoff >= p.sigma)))
        return TMD_EINVAL;
    const double r = p.cutoff + p.skin;
    if (!(r < 0.5 * L))
        return TMD_EBOX;
    const double ncd = floor(L / r);
    if (ncd > 1290.0)
        return TMD_EINVAL;
    B = Box{};
    B.atom_off = int32_t(atom_off);
    B.n = int32_t(n);
    B.nc = int32_t(ncd);  // >= 2 because r < L/2
    B.L = L;
    B.halfL = 0.5 * L;
    B.halfL2 = B.halfL * B.halfL;
    B.invL = 1.0 / L;
    B.side = L / B.nc;
    B.hside = 0.5 * B.side;
    B.rc2 = p.cutoff * p.cutoff;
    B.rl2 = r * r;
    set_lj(B, p.epsilon, p.sigma);
    B.h = 0.5 * p.dt / p.mass;
    B.dt = p.dt;
    B.mass = p.mass;
    B.sd_k = p.stiffness;
    B.sd_g = p.damping;
    B.sd_sig = p.sigma;
    B.sd_sig2 = p.sigma * p.sigma;
    return TMD_OK;
}

tmd_status create_impl(int32_t nbox, const int64_t *n_atoms, const double *lengths, const tmd_params *params,
                       tmd_system **out) {
    if (!out)
        return TMD_EINVAL;
    *out = nullptr;
    if (nbox < 1 || !n_atoms || !lengths || !params)
        return TMD_EINVAL;
    int64_t total = 0;
    std::vector<Box> boxes;
    try {
        boxes.resize(size_t(nbox));
    } catch (...) {
        return TMD_EINVAL;
    }
    for (int32_t k = 0; k < nbox; ++k) {
        const tmd_params &p = params[k];
        if (p.rebuild_every != params[0].rebuild_every || p.max_neighbors != params[0].max_neighbors ||
            p.model != params[0].model)
            return TMD_EINVAL;
        const tmd_status st = make_box(p, n_atoms[k], lengths[k], total, boxes[size_t(k)]);
        if (st != TMD_OK)
            return st;
        total += n_atoms[k];
        if (total > kMaxAtoms)
            return TMD_EINVAL;
    }
    tmd_system *s = new (std::nothrow) tmd_system();
    if (!s)
        return TMD_EINVAL;
    try {
        s->boxes = boxes;
        s->rebuild_every = params[0].rebuild_every;
        Dims &d = s->d;
        d.nt = int32_t(total);
        d.ntp = round_up(d.nt + 1, 256);  // slot nt holds the NaN sentinel atom
        d.nbox = nbox;
        d.maxnb = params[0].max_neighbors;
        d.nchunk = (d.maxnb + 3) / 4 + 1;  // one spare chunk of sentinel padding
        d.model = params[0].model;
        if (int64_t(d.ntp) * d.maxnb > (int64_t(1) << 40)) {
            delete s;
            return TMD_EINVAL;
        }
        s->atom_box.resize(size_t(d.ntp), nbox - 1);
        for (int32_t k = 0; k < nbox; ++k) {
            const Box &B = boxes[size_t(k)];
            std::fill(s->atom_box.begin() + B.atom_off, s->atom_box.begin() + B.atom_off + B.n, k);
        }
        // the workspace holds the tables of either block edge
        if (!layout_blocks(s, 3)) {
            delete s;
            return TMD_EINVAL;
        }
        Dims big = d;
        if (!layout_blocks(s, 2)) {
            delete s;
            return TMD_EINVAL;
        }
        big.nblk = std::max(big.nblk, d.nblk);
        big.ncs = std::max(big.ncs, d.ncs);
        s->dmax = big;
        const int E = default_edge(s->boxes.data(), nbox);
        if (E != 2)
            layout_blocks(s, E);
        s->ws_need = carve(s->dmax, nullptr, nullptr);
    } catch (...) {
        delete s;
        return TMD_EINVAL;
    }
    *out = s;
    return TMD_OK;
}

// One rebuild interval's list as the forward pass built it, kept for the
// reverse sweep, which then neither reloads nor rebins the interval's
// checkpoint: the interval's first positions (sorted order, with the NaN
// sentinel at slot nt), its atom order, and the list with its counts and
// neighborhood tables.
struct AdjList {
    Pos x;
    int32_t *orig, *cnt, *nbr, *hood;
};

// Carve one AdjList from base (sizes for dims d); with base == nullptr only
// the size is computed.
size_t carve_adj_list(const Dims &d, char *base, AdjList *out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    const size_t np = size_t(d.ntp);
    AdjList l{};
    l.x.x = (double *)take(np * 8);
    l.x.y = (double *)take(np * 8);
    l.x.z = (double *)take(np * 8);
    l.orig = (int32_t *)take(np * 4);
    l.cnt = (int32_t *)take(np * 4);
    l.nbr = (int32_t *)take(np * size_t(d.nchunk) * 4 * 4);
    l.hood = (int32_t *)take(size_t(d.nblk) * kHoodWords * 4);
    if (out)
        *out = l;
    return off;
}

// Adjoint workspace: checkpoints of (x, v) in original order at every
// rebuild step of the recorded run plus its final state, the positions of
// every step in the sorted order of its rebuild interval, each interval's
// list (AdjList), the cotangents and the parameter gradient accumulators.
struct AdjBuf {
    double *ckpt;   // [(nseg + 1) * 6 * nt]
    double *traj;   // [(nsteps + 1) * 3 * ntp]: slot k holds x_k (slot 0 unused)
    char *lists;    // nseg AdjLists of list_bytes each
    size_t list_bytes;
    Pos lx, wa, wb; // sorted order, ntp each
    double *lo;     // [6 * nt] cotangents in original order
    double *partials;
    double *acc;    // [2 * nbox]
};

size_t carve_adj(const Dims &d, int32_t R, int32_t nsteps, char *base, AdjBuf *out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    const size_t nt = size_t(d.nt), np = size_t(d.ntp);
    const int32_t nseg = (nsteps + R - 1) / R;
    AdjBuf a{};
    a.ckpt = (double *)take(size_t(nseg + 1) * 6 * nt * 8);
    a.traj = (double *)take(size_t(nsteps + 1) * 3 * np * 8);
    a.list_bytes = carve_adj_list(d, nullptr, nullptr);
    a.lists = take(size_t(nseg) * a.list_bytes);
    Pos *ps[3] = {&a.lx, &a.wa, &a.wb};
    for (Pos *p : ps) {
        p->x = (double *)take(np * 8);
        p->y = (double *)take(np * 8);
        p->z = (double *)take(np * 8);
    }
    a.lo = (double *)take(6 * nt * 8);
    a.partials = (double *)take(size_t(d.nblk) * kMaxParts * kPartialStride * 8);
    a.acc = (double *)take(size_t(d.nbox) * 2 * 8);
    if (out)
        *out = a;
    return off;
}

// Per-workgroup LDS limit of the current device.
hipError_t device_lds_limit(int &max_lds) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    return e;
}

// The adjoint kernel stages 48 bytes per atom (twice the 24 of the other
// block kernels): lower the capacity until its copy plus the static LDS of
// a block kernel fit the device's per-workgroup limit.  True if lowered.
bool fit_cap(Dims &d, int max_lds) {
    if (2 * hood_lds_bytes(d.cap) + size_t(kStaticLds) <= size_t(max_lds))
        return false;
    const int fit = int((size_t(max_lds) - size_t(kStaticLds)) / 48) - 2 - kHoodPad;
    d.cap = std::max(64, fit / 64 * 64);
    d.rcap = std::min(d.rcap, d.cap);  // the reaction sums then fit beside the copy too
    return true;
}

tmd_status upload_tables(tmd_system *s, hipStream_t hs) {
    hipError_t e = hipMemcpyAsync(s->b.boxes, s->boxes.data(), s->boxes.size() * sizeof(Box), hipMemcpyHostToDevice,
                                  hs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->b.blk_box, s->blk_box.data(), s->blk_box.size() * 4, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->b.atom_box, s->atom_box.data(), s->atom_box.size() * 4, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess)
        s->tables_dirty = false;
    if (e == hipSuccess && !s->prepared) {
        int max_lds = 0;
        e = device_lds_limit(max_lds);
        if (e == hipSuccess && fit_cap(s->d, max_lds))
            s->list_valid = s->force_valid = false;
        if (e == hipSuccess)
            e = prepare_kernels(max_lds - kStaticLds);
        s->prepared = (e == hipSuccess);
    }
    return e == hipSuccess ? TMD_OK : hip_fail(s, e, "table upload");
}

// What a captured interval bakes in: launch parameters, buffers, the copies
// the state starts in, whether the cell counts start at zero, the interval.
std::vector<unsigned char> seg_key(const tmd_system *s) {
    std::vector<unsigned char> k(sizeof(Dims) + sizeof(Buffers) + sizeof(Cursor) + 2 * sizeof(int32_t));
    unsigned char *p = k.data();
    std::memcpy(p, &s->d, sizeof(Dims));
    p += sizeof(Dims);
    std::memcpy(p, &s->b, sizeof(Buffers));
    p += sizeof(Buffers);
    std::memcpy(p, &s->cur, sizeof(Cursor));
    p += sizeof(Cursor);
    const int32_t extra[2] = {s->counts_clear ? 1 : 0, s->rebuild_every};
    std::memcpy(p, extra, sizeof(extra));
    return k;
}

void drop_segs(tmd_system *s) {
    for (auto &g : s->segs)
        (void)hipGraphExecDestroy(g.exec);
    s->segs.clear();
}

// After a force launch that kicked velocities: the Spring-Dashpot model
// wrote them to the other half.
void kicked(tmd_system *s) {
    if (s->d.model == TMD_MODEL_SPRING_DASHPOT)
        s->cur.v = 1 - s->cur.v;
}

// One rebuild interval of tmd_integrate's loop, starting right after a step
// whose number is a multiple of the interval: interval - 1 fused steps, the
// rebuild, and the fused step after it.
tmd_status enqueue_interval(tmd_system *s, hipStream_t hs) {
    for (int32_t k = 1; k <= s->rebuild_every; ++k) {
        if (k == s->rebuild_every) {
            const tmd_status st = rebuild(s, hs);
            if (st != TMD_OK)
                return st;
        }
        const hipError_t e = launch_force(s->d, s->b, s->cur, 2, false, hs);
        if (e != hipSuccess)
            return hip_fail(s, e, "force");
        s->cur.x = 1 - s->cur.x;
        kicked(s);
    }
    return TMD_OK;
}

// enqueue_interval() as one graph launch on hs: replayed when an interval
// with the same key was captured before, else captured on the system's own
// stream, instantiated and launched.  The host-side state advances as the
// eager path's would.
tmd_status run_interval(tmd_system *s, hipStream_t hs) {
    if (s->tables_dirty || !s->prepared) {
        const tmd_status u = upload_tables(s, hs);  // never inside a capture
        if (u != TMD_OK)
            return u;
    }
    const std::vector<unsigned char> key = seg_key(s);
    for (auto &g : s->segs)
        if (g.key == key) {
            const hipError_t e = hipGraphLaunch(g.exec, hs);
            if (e != hipSuccess)
                return hip_fail(s, e, "graph launch");
            s->graph_launches++;
            s->cur = g.cur_after;
            s->counts_clear = g.counts_clear_after;
            s->list_valid = true;
            s->force_valid = false;
            s->gen++;
            return TMD_OK;
        }
    if (s->segs.size() >= 2)
        drop_segs(s);  // parameters or buffers changed: the old graphs are stale
    hipError_t e = hipSuccess;
    if (!s->cap_stream)
        e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return hip_fail(s, e, "graph capture");
    const Cursor cur0 = s->cur;
    const bool clear0 = s->counts_clear, list0 = s->list_valid, force0 = s->force_valid;
    const tmd_status st = enqueue_interval(s, s->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s->cap_stream, &graph);
    tmd_system::Seg g;
    g.key = key;
    g.cur_after = s->cur;
    g.counts_clear_after = s->counts_clear;
    if (st == TMD_OK && e == hipSuccess)
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (graph)
        (void)hipGraphDestroy(graph);
    if (st != TMD_OK || e != hipSuccess) {
        // nothing ran: put the host-side state back
        s->cur = cur0;
        s->counts_clear = clear0;
        s->list_valid = list0;
        s->force_valid = force0;
        if (g.exec)
            (void)hipGraphExecDestroy(g.exec);
        return st != TMD_OK ? st : hip_fail(s, e, "graph capture");
    }
    e = hipGraphLaunch(g.exec, hs);
    s->segs.push_back(std::move(g));
    s->graph_captures++;
    if (e == hipSuccess)
        s->graph_launches++;
    return e == hipSuccess ? TMD_OK : hip_fail(s, e, "graph launch");
}

// Device memory of tmd_compute_forces_static: every GPU the library runs
// on holds its own copy of this array until the process ends.  Host code
// never uses the symbol's own address (a host-side stand-in): each device's
// address comes from hipGetSymbolAddress with that device current.
static __device__ __align__(256) unsigned char scratch[TMD_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct StaticDevice {
    bool ready = false;
    void *ptr = nullptr;  // this device's copy of `scratch`
    int max_lds = 0;      // per-workgroup LDS limit
};

std::mutex g_static_mu;
StaticDevice g_static[kMaxDevices];

// Once per device, with it current: the array's device address and the
// block kernels' dynamic-LDS attribute.
tmd_status static_device(StaticDevice &out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return TMD_EHIP;
    if (dev < 0 || dev >= kMaxDevices)
        return TMD_EINVAL;
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticDevice &sd = g_static[dev];
    if (!sd.ready) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return TMD_EHIP;
        int max_lds = 0;
        if (device_lds_limit(max_lds) != hipSuccess || prepare_kernels(max_lds - kStaticLds) != hipSuccess)
            return TMD_EHIP;
        sd.ptr = p;
        sd.max_lds = max_lds;
        sd.ready = true;
    }
    out = sd;
    return TMD_OK;
}

}  // namespace

extern "C" {

const char *tmd_status_string(tmd_status st) {
    switch (st) {
    case TMD_OK: return "ok";
    case TMD_EINVAL: return "invalid argument";
    case TMD_EBOX: return "cutoff + skin must be smaller than half the box length";
    case TMD_ESTATE: return "invalid call order";
    case TMD_ENBR_OVERFLOW: return "neighbor list capacity exceeded";
    case TMD_ENONFINITE: return "non-finite position, velocity or force";
    case TMD_EWORKSPACE: return "workspace too small or misaligned";
    case TMD_EHIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *tmd_last_error(const tmd_system *s) { return s ? s->err.c_str() : "NULL system"; }

tmd_status tmd_create(const tmd_params *p, int64_t n_atoms, double L, tmd_system **out) {
    return create_impl(1, &n_atoms, &L, p, out);
}

tmd_status tmd_create_batch(int32_t n_boxes, const int64_t *n_atoms, const double *box_lengths,
                            const tmd_params *params, tmd_system **out) {
    return create_impl(n_boxes, n_atoms, box_lengths, params, out);
}

tmd_status tmd_workspace_size(const tmd_system *s, size_t *bytes) {
    if (!s || !bytes)
        return TMD_EINVAL;
    *bytes = s->ws_need;
    return TMD_OK;
}

tmd_status tmd_bind_workspace(tmd_system *s, void *dev, size_t bytes) {
    if (!s || !dev)
        return TMD_EINVAL;
    if (bytes < s->ws_need || (reinterpret_cast<uintptr_t>(dev) % kAlign) != 0)
        return fail(s, TMD_EWORKSPACE, "workspace must be 256-byte aligned and at least tmd_workspace_size bytes");
    carve(s->dmax, static_cast<char *>(dev), &s->b);
    s->counts_clear = false;
    s->tables_dirty = true;
    s->bound = true;
    s->gen++;
    s->have_state = s->list_valid = s->force_valid = false;
    s->cur = Cursor{};
    return TMD_OK;
}

tmd_status tmd_set_state(tmd_system *s, const double *const pos[3], const double *const vel[3], int64_t step,
                         tmd_stream stream) {
    tmd_status st = check_ready(s, false);
    if (st != TMD_OK)
        return st;
    if (!pos || !vel || !pos[0] || !pos[1] || !pos[2] || !vel[0] || !vel[1] || !vel[2] || step < 0)
        return fail(s, TMD_EINVAL, "set_state: NULL array or negative step");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if ((st = upload_tables(s, hs)) != TMD_OK)
        return st;
    hipError_t e;
    {
        Timed t(s, TMD_T_COPY, hs);
        e = launch_fill_i32(s->b.err, 0, 16, hs);
        if (e == hipSuccess)
            e = launch_load_state(s->d, pos, vel, s->b, Cursor{}, hs);
    }
    if (e != hipSuccess)
        return hip_fail(s, e, "set_state");
    s->cur = Cursor{};
    s->step = step;
    s->have_state = true;
    s->gen++;
    s->list_valid = s->force_valid = false;
    return TMD_OK;
}

tmd_status tmd_build_neighbors(tmd_system *s, tmd_stream stream) {
    tmd_status st = check_ready(s, true);
    if (st != TMD_OK)
        return st;
    return rebuild(s, static_cast<hipStream_t>(stream));
}

tmd_status tmd_compute_forces(tmd_system *s, double *const f[3], double *ev, tmd_stream stream) {
    tmd_status st = check_ready(s, true);
    if (st != TMD_OK)
        return st;
    if (!s->list_valid)
        return fail(s, TMD_ESTATE, "compute_forces: no neighbor list built since the state was set");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e;
    {
        Timed t(s, TMD_T_FORCE, hs);
        e = launch_force(s->d, s->b, s->cur, 0, ev != nullptr, hs);
    }
    if (e != hipSuccess)
        return hip_fail(s, e, "force");
    s->force_valid = true;
    if (ev) {
        Timed t(s, TMD_T_THERMO, hs);
        e = launch_reduce(s->d, s->b, ev, 2, hs);
        if (e != hipSuccess)
            return hip_fail(s, e, "reduce");
    }
    if (f && (f[0] || f[1] || f[2])) {
        Timed t(s, TMD_T_COPY, hs);
        e = launch_unload(s->d, s->b.fx, s->b.fy, s->b.fz, s->b.orig[s->cur.o], f, hs);
        if (e != hipSuccess)
            return hip_fail(s, e, "force unload");
    }
    return TMD_OK;
}

tmd_status tmd_integrate(tmd_system *s, int32_t n_steps, int32_t thermo_every, double *thermo, tmd_stream stream) {
    tmd_status st = check_ready(s, true);
    if (st != TMD_OK)
        return st;
    if (n_steps < 0 || thermo_every < 0 || (thermo_every > 0 && !thermo))
        return fail(s, TMD_EINVAL, "integrate: negative count or thermo_every > 0 without a thermo buffer");
    if (n_steps == 0)
        return TMD_OK;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (!s->list_valid && (st = rebuild(s, hs)) != TMD_OK)
        return st;
    if (!s->force_valid) {
        Timed t(s, TMD_T_FORCE, hs);
        e = launch_force(s->d, s->b, s->cur, 0, false, hs);
        if (e != hipSuccess)
            return hip_fail(s, e, "force");
        s->force_valid = true;
    }
    {
        Timed t(s, TMD_T_DRIFT, hs);
        e = launch_drift(s->d, s->b, s->cur, hs);
    }
    if (e != hipSuccess)
        return hip_fail(s, e, "drift");
    s->cur.x = 1 - s->cur.x;
    s->force_valid = false;
    const int64_t rb = s->rebuild_every;
    const int64_t row_stride = int64_t(s->d.nbox) * 5;
    TimedRun run(s, TMD_T_FORCE, hs);
    const bool graphs = s->graphs && thermo_every == 0 && !s->timing;
    for (int32_t k = 1; k <= n_steps; ++k) {
        const int64_t stepk = s->step + k;
        if (graphs && (stepk - 1) % rb == 0 && int64_t(k) - 1 + rb <= int64_t(n_steps) - 1) {
            // a whole rebuild interval before the last step: one graph launch
            if ((st = run_interval(s, hs)) != TMD_OK)
                return st;
            k += int32_t(rb) - 1;
            continue;
        }
        if (stepk % rb == 0) {
            run.close();
            if ((st = rebuild(s, hs)) != TMD_OK)
                return st;
        }
        const bool th = thermo_every > 0 && (k % thermo_every) == 0;
        const int mode = (k < n_steps) ? 2 : 1;
        run.add();
        e = launch_force(s->d, s->b, s->cur, mode, th, hs);
        if (e != hipSuccess)
            return hip_fail(s, e, "force");
        if (mode == 2)
            s->cur.x = 1 - s->cur.x;
        kicked(s);
        if (th) {
            run.close();
            Timed t(s, TMD_T_THERMO, hs);
            e = launch_reduce(s->d, s->b, thermo + int64_t(k / thermo_every - 1) * row_stride, 5, hs);
            if (e != hipSuccess)
                return hip_fail(s, e, "reduce");
        }
    }
    s->force_valid = true;
    s->step += n_steps;
    s->gen++;
    return TMD_OK;
}

tmd_status tmd_get_state(const tmd_system *cs, double *const pos[3], double *const vel[3], int64_t *step,
                         tmd_stream stream) {
    tmd_system *s = const_cast<tmd_system *>(cs);
    tmd_status st = check_ready(s, true);
    if (st != TMD_OK)
        return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const int c = s->cur.x, o = s->cur.o;
    Timed t(s, TMD_T_COPY, hs);
    if (pos) {
        hipError_t e = launch_unload_pos(s->d, s->b, s->b.pos(c), s->b.orig[o], pos, hs);
        if (e != hipSuccess)
            return hip_fail(s, e, "get_state");
    }
    if (vel) {
        const int v = s->cur.v;
        hipError_t e = launch_unload(s->d, s->b.vx[v], s->b.vy[v], s->b.vz[v], s->b.orig[o], vel, hs);
        if (e != hipSuccess)
            return hip_fail(s, e, "get_state");
    }
    if (step)
        *step = s->step;
    return TMD_OK;
}

tmd_status tmd_get_neighbors(const tmd_system *cs, int32_t *counts, int32_t *ids, int64_t capacity,
                             tmd_stream stream) {
    tmd_system *s = const_cast<tmd_system *>(cs);
    tmd_status st = check_ready(s, true);
    if (st != TMD_OK)
        return st;
    if (!counts || (ids && capacity < int64_t(s->d.nt) * s->d.maxnb))
        return fail(s, TMD_EINVAL, "get_neighbors: NULL counts or capacity below n_atoms * max_neighbors");
    if (!s->list_valid)
        return fail(s, TMD_ESTATE, "get_neighbors: no list built since the state was set");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    Timed t(s, TMD_T_COPY, hs);
    hipError_t e = launch_export_neighbors(s->d, s->b, s->cur, counts, ids, hs);
    return e == hipSuccess ? TMD_OK : hip_fail(s, e, "get_neighbors");
}

tmd_status tmd_sync(tmd_system *s, tmd_stream stream) {
    tmd_status st = check_ready(s, false);
    if (st != TMD_OK)
        return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    int32_t w[2] = {0, 0};
    hipError_t e = hipSuccess;
    if (s->have_state)
        e = hipMemcpyAsync(w, s->b.err, sizeof(w), hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess)
        e = hipStreamSynchronize(hs);
    if (e != hipSuccess)
        return hip_fail(s, e, "sync");
    if (w[0] & kErrNonFinite)
        return fail(s, TMD_ENONFINITE, "a position, velocity or force became NaN/Inf (coincident atoms?)");
    if (w[0] & kErrOverflow)
        return fail(s, TMD_ENBR_OVERFLOW, "an atom has " + std::to_string(w[1]) + " list entries, max_neighbors is " +
                                              std::to_string(s->d.maxnb));
    if (w[0] & kErrOutOfBox)
        return fail(s, TMD_EINVAL, "set_state: a coordinate lies outside [-L, 2L)");
    if (w[0] & kErrLdsLayout)
        return fail(s, TMD_EHIP, "internal: the force kernel's dynamic LDS does not start at address 0");
    return TMD_OK;
}

tmd_status tmd_get_info(const tmd_system *s, tmd_info *info) {
    if (!s || !info)
        return TMD_EINVAL;
    int64_t cells = 0;
    for (const Box &B : s->boxes)
        cells += int64_t(B.nc) * B.nc * B.nc;
    info->n_atoms = s->d.nt;
    info->n_padded = s->d.ntp;
    info->cells_per_axis = s->boxes[0].nc;
    info->max_neighbors = s->d.maxnb;
    info->n_cells = cells;
    info->workspace_bytes = s->ws_need;
    info->step = s->step;
    info->n_boxes = s->d.nbox;
    info->n_blocks = s->d.nblk;
    info->block_threads = s->d.threads;
    info->lds_atoms = s->d.cap;
    info->block_edge = s->d.edge;
    info->block_parts = s->d.parts;
    info->lanes_per_atom = s->d.lpa;
    info->build_threads = s->d.bthreads;
    info->build_lanes = s->d.blanes;
    info->graph_captures = s->graph_captures;
    info->graph_launches = s->graph_launches;
    info->half_list = s->d.half;
    info->layout = s->d.layout;
    return TMD_OK;
}

tmd_status tmd_set_schedule(tmd_system *s, int32_t threads, int32_t lds_atoms, int32_t block_edge,
                            int32_t block_parts, int32_t lanes_per_atom, int32_t build_threads, int32_t build_lanes) {
    if (!s || threads < 0 || threads > kMaxThreads || threads % 64 != 0 || build_threads < 0 ||
        (build_lanes != 0 && build_lanes != 1 && build_lanes != 2) ||
        build_threads > kMaxThreads || build_threads % 64 != 0 || lds_atoms < 0 || lds_atoms > kMaxCap ||
        lds_atoms % 64 != 0 || (block_edge != 0 && block_edge != 2 && block_edge != 3) ||
        (block_parts != 0 && block_parts != 1 && block_parts != 2 && block_parts != 4) ||
        (lanes_per_atom != 0 && lanes_per_atom != 1 && lanes_per_atom != 2 && lanes_per_atom != 4) ||
        (lanes_per_atom > 1 && s->d.model == 1) || (s->d.half && (block_parts > 1 || lanes_per_atom > 1)))
        return TMD_EINVAL;
    if (block_edge != 0 && block_edge != s->d.edge) {
        layout_blocks(s, block_edge);  // resets threads and capacity to that edge's defaults
        s->list_valid = s->force_valid = false;
        s->gen++;
    }
    if (block_parts != 0 && block_parts != s->d.parts) {
        s->d.parts = block_parts;  // the list does not depend on it
        s->d.threads = default_threads(s->d, s->d.lpa);
        s->d.bthreads = default_threads(s->d, s->d.blanes);
    }
    if (build_lanes != 0 && build_lanes != s->d.blanes) {
        s->d.blanes = build_lanes;  // nor on this: both lane counts write the same list
        s->d.bthreads = default_threads(s->d, s->d.blanes);
    }
    if (lanes_per_atom != 0 && lanes_per_atom != s->d.lpa) {
        s->d.lpa = lanes_per_atom;  // nor on this
        s->d.threads = default_threads(s->d, s->d.lpa);
        s->force_valid = false;      // forces are summed in another order
    }
    if (threads > 0)
        s->d.threads = threads;
    if (build_threads > 0)
        s->d.bthreads = build_threads;
    if (lds_atoms > 0 && lds_atoms != s->d.cap) {
        s->d.cap = lds_atoms;
        if (s->d.half)
            s->d.rcap = std::min(s->d.rcap, lds_atoms);
        s->prepared = false;  // LDS attribute of the block kernels must follow
        // the list encodes LDS slots only for neighborhoods that fit
        s->list_valid = s->force_valid = false;
        s->gen++;
    }
    return TMD_OK;
}

static_assert(TMD_LAYOUT_SOA == kLayoutSoA && TMD_LAYOUT_AOS == kLayoutAoS && TMD_LAYOUT_AOSOA == kLayoutAoSoA,
              "public and internal layout codes agree");

// Convert the current positions to `layout` (the other position half takes
// them, and the sentinel in both halves follows).
static tmd_status relayout(tmd_system *s, int32_t layout, hipStream_t hs) {
    if (layout == s->d.layout)
        return TMD_OK;
    if (s->have_state) {
        const hipError_t e = launch_relayout(s->d, s->b, s->cur, layout, hs);
        if (e != hipSuccess)
            return hip_fail(s, e, "set_layout");
        s->cur.x = 1 - s->cur.x;
    }
    s->d.layout = layout;
    s->gen++;  // a recorded adjoint run reads the state's positions as SoA
    return TMD_OK;
}

tmd_status tmd_set_layout(tmd_system *s, int32_t layout, tmd_stream stream) {
    if (!s || (layout != kLayoutSoA && layout != kLayoutAoS && layout != kLayoutAoSoA))
        return TMD_EINVAL;
    if (layout != kLayoutSoA && s->d.model != TMD_MODEL_LJ)
        return fail(s, TMD_EINVAL, "set_layout: the Spring-Dashpot model keeps SoA positions");
    return relayout(s, layout, static_cast<hipStream_t>(stream));
}

tmd_status tmd_set_half_list(tmd_system *s, int32_t half) {
    if (!s || (half != 0 && half != 1))
        return TMD_EINVAL;
    if (half && (s->d.model != TMD_MODEL_LJ || s->d.parts != 1 || s->d.lpa != 1))
        return TMD_EINVAL;
    if (half != s->d.half) {
        s->d.half = half;
        // the LDS split between staging and reaction sums follows; threads
        // and capacity return to the edge's defaults
        layout_blocks(s, s->d.edge);
        s->list_valid = s->force_valid = false;  // another list, forces summed in another order
        s->gen++;
    }
    return TMD_OK;
}

// Mean duration (ms) of `repeats` launches of the kernel an integrate step
// runs (force sum, two kicks and the drift) on the current list.  They read
// the current positions and a copy of the velocities in the spare velocity
// buffer, and write the spare position buffer: the state is not changed.
static hipError_t time_force(tmd_system *s, int32_t repeats, hipStream_t hs, hipEvent_t a, hipEvent_t b, float &ms) {
    Buffers &bf = s->b;
    const int c = s->cur.x, o = s->cur.v;
    // the Spring-Dashpot kernel would kick into the state's own velocity
    // half: time its force-only launch (the same pair work)
    const int mode = s->d.model == TMD_MODEL_SPRING_DASHPOT ? 0 : 2;
    const size_t bytes = size_t(s->d.nt) * sizeof(double);
    hipError_t e = hipMemcpyAsync(bf.vx[1 - o], bf.vx[o], bytes, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bf.vy[1 - o], bf.vy[o], bytes, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bf.vz[1 - o], bf.vz[o], bytes, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess)  // warm-up
        e = launch_force_at(s->d, bf, bf.pos(c), bf.pos(1 - c), 1 - o, mode, false, hs);
    if (e == hipSuccess)
        e = hipEventRecord(a, hs);
    for (int32_t r = 0; r < repeats && e == hipSuccess; ++r)
        e = launch_force_at(s->d, bf, bf.pos(c), bf.pos(1 - c), 1 - o, mode, false, hs);
    if (e == hipSuccess)
        e = hipEventRecord(b, hs);
    if (e == hipSuccess)
        e = hipEventSynchronize(b);
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, a, b);
    ms /= float(repeats);
    return e;
}

// Average time of one list build at the current schedule (it rewrites the
// same list: positions and binning are unchanged).
static hipError_t time_build(tmd_system *s, int32_t repeats, hipStream_t hs, hipEvent_t a, hipEvent_t b, float &ms) {
    hipError_t e = hipEventRecord(a, hs);
    for (int32_t r = 0; r < repeats && e == hipSuccess; ++r)
        e = launch_build(s->d, s->b, s->cur, hs);
    if (e == hipSuccess)
        e = hipEventRecord(b, hs);
    if (e == hipSuccess)
        e = hipEventSynchronize(b);
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, a, b);
    ms /= float(repeats);
    return e;
}

tmd_status tmd_autotune(tmd_system *s, int32_t repeats, int32_t flags, tmd_stream stream) {
    tmd_status st = check_ready(s, true);
    if (st != TMD_OK)
        return st;
    if (repeats < 1 || (flags & ~TMD_TUNE_ADJOINT) != 0)
        return fail(s, TMD_EINVAL, "autotune: repeats < 1 or unknown flags");
    const bool for_adjoint = (flags & TMD_TUNE_ADJOINT) != 0;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    if (e != hipSuccess)
        return hip_fail(s, e, "autotune");
    float best = 1e30f;
    int32_t best_edge = s->d.edge, best_t = s->d.threads, best_p = s->d.parts, best_l = s->d.lpa,
            best_bt = s->d.bthreads, best_bl = s->d.blanes, best_h = s->d.half;
    // half lists (Lennard-Jones only) take one workgroup per block and one
    // lane per atom
    const int32_t hmax = s->d.model == TMD_MODEL_LJ && !for_adjoint ? 1 : 0;
    for (int32_t EH = 0; EH < (kMaxEdge - 1) * (hmax + 1) && e == hipSuccess; ++EH) {
        const int32_t E = 2 + EH / (hmax + 1), H = EH % (hmax + 1);
        s->d.half = H;
        layout_blocks(s, E);
        s->d.parts = 1;
        s->d.lpa = 1;
        s->list_valid = s->force_valid = false;
        if ((st = rebuild(s, hs)) != TMD_OK)
            break;
        for (int32_t P = 1; P <= (H ? 1 : kMaxParts) && e == hipSuccess; P *= 2) {
            s->d.parts = P;
            // the list build's lanes per atom and threads are tuned on their
            // own (the build and the force kernel share only the blocks)
            float mb = 1e30f;
            int32_t bt_best = s->d.bthreads, bl_best = s->d.blanes;
            for (int32_t BL = 1; BL <= 2 && e == hipSuccess; ++BL) {
                s->d.blanes = BL;
                const int32_t b0 = default_threads(s->d, BL);
                for (int32_t t = std::max(64, b0 - 128); t <= std::min(kMaxThreads, b0 + 128) && e == hipSuccess;
                     t += 64) {
                    s->d.bthreads = t;
                    float m = 0.0f;
                    e = time_build(s, repeats, hs, a, b, m);
                    // builds timed back to back find their data in the caches; in
                    // a run each build follows binning and many force launches,
                    // and there more threads stage the cold neighborhood faster:
                    // within 5% the larger workgroup wins
                    if (e == hipSuccess && (m < mb || (m < 1.05f * mb && BL == bl_best && t > bt_best))) {
                        mb = std::min(mb, m);
                        bt_best = t;
                        bl_best = BL;
                    }
                }
            }
            s->d.bthreads = bt_best;
            s->d.blanes = bl_best;
            for (int32_t Lp = 1; Lp <= (s->d.model == 1 || H ? 1 : 4) && e == hipSuccess; Lp *= 2) {
                s->d.lpa = Lp;
                // from one lane group per mean block atom (in whole
                // wavefronts) up to two wavefronts more: fewer threads put
                // most blocks through a partial second pass, which launches
                // timed back to back on unchanged inputs can rank first
                // although it is slower in a run
                const int32_t t0 = default_threads(s->d, Lp);
                // within 4% the larger workgroup of this sweep wins: its
                // extra wavefronts stage the neighborhood faster, which
                // launches timed back to back (inputs in the caches) show
                // less than a run does (131k atoms: 192 threads can time
                // level with 320 here, and run 5% slower)
                float lbest = 1e30f;
                int32_t lt = t0;
                for (int32_t t = t0; t <= std::min(kMaxThreads, t0 + 128) && e == hipSuccess; t += 64) {
                    s->d.threads = t;
                    // cost per step: one force evaluation plus the list build's share
                    float ms = 0.0f;
                    e = time_force(s, repeats, hs, a, b, ms);
                    ms += mb / float(s->rebuild_every);
                    if (e == hipSuccess && ms < 1.04f * lbest) {
                        lbest = std::min(lbest, ms);
                        lt = t;
                    }
                }
                if (e == hipSuccess && lbest < best) {
                    best = lbest;
                    best_edge = E;
                    best_t = lt;
                    best_p = P;
                    best_l = Lp;
                    best_bt = bt_best;
                    best_bl = bl_best;
                    best_h = H;
                }
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != TMD_OK)
        return st;
    if (e != hipSuccess)
        return hip_fail(s, e, "autotune");
    s->d.half = best_h;
    layout_blocks(s, best_edge);
    s->d.parts = best_p;
    s->d.lpa = best_l;
    s->d.threads = best_t;
    s->d.bthreads = best_bt;
    s->d.blanes = best_bl;
    s->list_valid = s->force_valid = false;
    if ((st = rebuild(s, hs)) != TMD_OK)
        return st;
    // the position layout, at the chosen schedule: a list build and the
    // step kernel read positions (binning does too, once per rebuild, as
    // the build)
    if (for_adjoint && (st = relayout(s, kLayoutSoA, hs)) != TMD_OK)
        return st;
    if (s->d.model == TMD_MODEL_LJ && !for_adjoint) {
        e = hipEventCreate(&a);
        if (e == hipSuccess)
            e = hipEventCreate(&b);
        const int32_t start = s->d.layout;
        float lbest = 1e30f;
        int32_t best_lay = start;
        for (int32_t lay = 0; lay < 3 && e == hipSuccess && st == TMD_OK; ++lay) {
            if ((st = relayout(s, lay, hs)) != TMD_OK)
                break;
            float mb = 0.0f, mf = 0.0f;
            e = time_build(s, repeats, hs, a, b, mb);
            if (e == hipSuccess)
                e = time_force(s, repeats, hs, a, b, mf);
            const float ms = mf + mb / float(s->rebuild_every);
            // within 1% the earlier (SoA first) layout stays
            if (e == hipSuccess && ms < 0.99f * lbest) {
                lbest = ms;
                best_lay = lay;
            }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (st == TMD_OK && e == hipSuccess)
            st = relayout(s, best_lay, hs);
        if (st != TMD_OK)
            return st;
        if (e != hipSuccess)
            return hip_fail(s, e, "autotune");
    }
    return TMD_OK;
}

tmd_status tmd_set_lj_params(tmd_system *s, const double *epsilon, const double *sigma, tmd_stream stream) {
    tmd_status st = check_ready(s, false);
    if (st != TMD_OK)
        return st;
    if (!epsilon || !sigma)
        return fail(s, TMD_EINVAL, "set_lj_params: NULL array");
    if (s->d.model != TMD_MODEL_LJ)
        return fail(s, TMD_EINVAL, "set_lj_params: the system uses the Spring-Dashpot model");
    for (int32_t k = 0; k < s->d.nbox; ++k)
        if (!positive(epsilon[k]) || !positive(sigma[k]))
            return fail(s, TMD_EINVAL, "set_lj_params: epsilon and sigma must be finite and positive");
    for (int32_t k = 0; k < s->d.nbox; ++k)
        set_lj(s->boxes[size_t(k)], epsilon[k], sigma[k]);
    hipError_t e = hipMemcpyAsync(s->b.boxes, s->boxes.data(), s->boxes.size() * sizeof(Box), hipMemcpyHostToDevice,
                                  static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(s, e, "set_lj_params");
    s->force_valid = false;
    s->gen++;
    return TMD_OK;
}

tmd_status tmd_adjoint_workspace_size(const tmd_system *s, int32_t n_steps, size_t *bytes) {
    if (!s || !bytes || n_steps < 1)
        return TMD_EINVAL;
    *bytes = carve_adj(s->dmax, s->rebuild_every, n_steps, nullptr, nullptr);
    return TMD_OK;
}

// The atom order and first positions of interval m into its AdjList (its
// list is built there in place).
static hipError_t save_adj_state(tmd_system *s, const AdjBuf &a, int32_t m, hipStream_t hs) {
    AdjList l{};
    carve_adj_list(s->dmax, a.lists + size_t(m) * a.list_bytes, &l);
    const Dims &d = s->d;
    const Buffers &b = s->b;
    const size_t np = size_t(d.ntp);
    const double *src[3] = {b.x[s->cur.x], b.y[s->cur.x], b.z[s->cur.x]};
    double *dst[3] = {l.x.x, l.x.y, l.x.z};
    hipError_t e = hipSuccess;
    for (int q = 0; q < 3 && e == hipSuccess; ++q)
        e = hipMemcpyAsync(dst[q], src[q], np * 8, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(l.orig, b.orig[s->cur.o], size_t(d.nt) * 4, hipMemcpyDeviceToDevice, hs);
    return e;
}

// While the forward pass runs, the system's list buffers (counts, list,
// neighborhood tables) are those of an interval's AdjList, so each
// interval's rebuild writes its list straight into the workspace; the
// system's own buffers come back when this goes out of scope (a run that
// ends there, on an error, while they are still redirected leaves no valid
// list or forces).
struct ListRedirect {
    tmd_system *s;
    int32_t *const cnt, *const nbr, *const hood;
    explicit ListRedirect(tmd_system *s_)
        : s(s_), cnt(s_->b.nbr_count), nbr(s_->b.nbr), hood(s_->b.hood_tab) {}
    ~ListRedirect() {
        if (s->b.nbr != nbr) {
            s->list_valid = false;
            s->force_valid = false;
        }
        restore();
    }
    void to(const AdjList &l) {
        Buffers &b = s->b;
        b.nbr_count = l.cnt;
        b.nbr = l.nbr;
        b.hood_tab = l.hood;
    }
    void restore() {
        Buffers &b = s->b;
        b.nbr_count = cnt;
        b.nbr = nbr;
        b.hood_tab = hood;
    }
};

tmd_status tmd_adjoint_forward(tmd_system *s, int32_t n_steps, void *ws, size_t bytes, tmd_stream stream) {
    tmd_status st = check_ready(s, true);
    if (st != TMD_OK)
        return st;
    if (n_steps < 1 || !ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 ||
        bytes < carve_adj(s->dmax, s->rebuild_every, n_steps, nullptr, nullptr))
        return fail(s, TMD_EINVAL, "adjoint_forward: n_steps < 1 or workspace missing, misaligned or too small");
    if (s->d.model != TMD_MODEL_LJ)
        return fail(s, TMD_EINVAL, "adjoint_forward: gradients are implemented for the Lennard-Jones model only");
    if (s->d.half)
        return fail(s, TMD_EINVAL, "adjoint_forward: the reverse pass needs full lists (tmd_set_half_list(0))");
    if (s->d.layout != kLayoutSoA)
        return fail(s, TMD_EINVAL, "adjoint_forward: the reverse pass needs TMD_LAYOUT_SOA positions");
    const int32_t R = s->rebuild_every;
    if (s->step % R != 0)
        return fail(s, TMD_ESTATE, "adjoint_forward: the step counter must be a multiple of rebuild_every");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    AdjBuf a{};
    carve_adj(s->dmax, R, n_steps, static_cast<char *>(ws), &a);
    const int32_t nseg = (n_steps + R - 1) / R;
    const size_t nt = size_t(s->d.nt), np = size_t(s->d.ntp);
    const int64_t step0 = s->step;
    Buffers &b = s->b;
    // every stored position buffer carries the NaN sentinel atom (slot nt)
    // that padding of 32-bit lists points at
    hipError_t e = launch_traj_sentinels(a.traj, np, s->d.nt, n_steps, hs);
    auto slot = [&](int32_t k) {
        double *t = a.traj + size_t(k) * 3 * np;
        return Pos{t, t + np, t + 2 * np};
    };
    // Each interval starts from its checkpoint, binned as the backward pass
    // will bin it (the same list and atom order), and runs the
    // velocity-Verlet steps of tmd_integrate with explicit output buffers:
    // x_{k+1} of every step goes to store slot k + 1, in the interval's
    // sorted order.  The interval's last step then finishes as tmd_integrate
    // finishes it (rebuild at a rebuild step, force and closing kick).  The
    // first interval reloads its checkpoint and bins it; every later one
    // starts where the previous one ended, which already is that state:
    // binning orders atoms by cell and original id whatever their order
    // before, and wraps positions into the box (wrapping twice changes
    // nothing), so a reload would give the same positions, order, list and
    // forces bit for bit.
    ListRedirect redirect(s);
    auto list_of = [&](int32_t m) {
        AdjList l{};
        carve_adj_list(s->dmax, a.lists + size_t(m) * a.list_bytes, &l);
        return l;
    };
    bool rebuilt_last = false;
    for (int32_t m = 0; m < nseg && e == hipSuccess; ++m) {
        const int32_t k_lo = m * R, len = std::min(R, n_steps - k_lo);
        double *c = a.ckpt + size_t(m) * 6 * nt;
        double *const po[3] = {c, c + nt, c + 2 * nt};
        double *const vo[3] = {c + 3 * nt, c + 4 * nt, c + 5 * nt};
        if ((st = tmd_get_state(s, po, vo, nullptr, stream)) != TMD_OK)
            return st;
        if (m == 0) {
            const double *const pi[3] = {po[0], po[1], po[2]};
            const double *const vi[3] = {vo[0], vo[1], vo[2]};
            e = launch_load_state(s->d, pi, vi, b, Cursor{}, hs);
            s->cur = Cursor{};
            redirect.to(list_of(0));
            if (e == hipSuccess && (st = rebuild(s, hs)) != TMD_OK)
                return st;
        }
        const int o = s->cur.v;
        const Pos x0 = b.pos(s->cur.x);
        auto traj = [&](int32_t j) { return j == 0 ? x0 : slot(k_lo + j); };
        if (e == hipSuccess)
            e = save_adj_state(s, a, m, hs);
        if (e == hipSuccess && m == 0)
            e = launch_force_at(s->d, b, x0, x0, o, 0, false, hs);
        if (e == hipSuccess)
            e = launch_drift_at(s->d, b, x0, traj(1), o, hs);
        for (int32_t j = 1; j < len && e == hipSuccess; ++j)
            e = launch_force_at(s->d, b, traj(j), traj(j + 1), o, 2, false, hs);
        // step k_lo + len: its positions become the system's
        const Pos xe = traj(len), xs = b.pos(s->cur.x);
        for (int q = 0; q < 3 && e == hipSuccess; ++q) {
            const double *src = q == 0 ? xe.x : (q == 1 ? xe.y : xe.z);
            double *dst = q == 0 ? xs.x : (q == 1 ? xs.y : xs.z);
            e = hipMemcpyAsync(dst, src, nt * sizeof(double), hipMemcpyDeviceToDevice, hs);
        }
        if (e == hipSuccess && (step0 + k_lo + len) % R == 0) {
            // the next interval's list (past the last interval: the system's)
            if (m + 1 < nseg)
                redirect.to(list_of(m + 1));
            else
                redirect.restore();
            if ((st = rebuild(s, hs)) != TMD_OK)
                return st;
            rebuilt_last = m + 1 == nseg;
        }
        if (e == hipSuccess)
            e = launch_force(s->d, b, s->cur, 1, false, hs);
        s->force_valid = true;
        s->step = step0 + k_lo + len;
    }
    // a run that ends between rebuilds keeps the last interval's list:
    // the system's own buffers take a copy
    if (e == hipSuccess && !rebuilt_last) {
        const AdjList l = list_of(nseg - 1);
        redirect.restore();
        e = hipMemcpyAsync(b.nbr_count, l.cnt, nt * 4, hipMemcpyDeviceToDevice, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.nbr, l.nbr, np * size_t(s->d.nchunk) * 16, hipMemcpyDeviceToDevice, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.hood_tab, l.hood, size_t(s->d.nblk) * kHoodWords * 4, hipMemcpyDeviceToDevice,
                               hs);
    }
    redirect.restore();
    if (e != hipSuccess)
        return hip_fail(s, e, "adjoint_forward");
    {
        double *c = a.ckpt + size_t(nseg) * 6 * nt;
        double *const po[3] = {c, c + nt, c + 2 * nt};
        double *const vo[3] = {c + 3 * nt, c + 4 * nt, c + 5 * nt};
        if ((st = tmd_get_state(s, po, vo, nullptr, stream)) != TMD_OK)
            return st;
    }
    s->gen++;
    s->adj.recorded = true;
    s->adj.step0 = step0;
    s->adj.nsteps = n_steps;
    s->adj.nseg = nseg;
    s->adj.ws = ws;
    s->adj.gen = ++s->gen;
    return TMD_OK;
}

tmd_status tmd_adjoint_backward(tmd_system *s, void *ws, size_t bytes, const double *const lam_x[3],
                                const double *const lam_v[3], double *const grad_x0[3], double *const grad_v0[3],
                                double *grad_eps, double *grad_sigma, tmd_stream stream) {
    tmd_status st = check_ready(s, true);
    if (st != TMD_OK)
        return st;
    if (!s->adj.recorded || ws != s->adj.ws || s->gen != s->adj.gen)
        return fail(s, TMD_ESTATE, "adjoint_backward: no forward run recorded in this workspace, or the state "
                                   "changed since");
    if (bytes < carve_adj(s->dmax, s->rebuild_every, s->adj.nsteps, nullptr, nullptr) || !lam_x || !lam_x[0] ||
        !lam_x[1] || !lam_x[2] || !grad_x0 || !grad_x0[0] || !grad_x0[1] || !grad_x0[2])
        return fail(s, TMD_EINVAL, "adjoint_backward: workspace too small or NULL cotangent / gradient array");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const int32_t R = s->rebuild_every, T = s->adj.nsteps, nseg = s->adj.nseg;
    const size_t nt = size_t(s->d.nt);
    AdjBuf a{};
    carve_adj(s->dmax, R, T, static_cast<char *>(ws), &a);
    Buffers &b = s->b;
    hipError_t e = launch_fill_f64(a.acc, 0.0, 2 * s->d.nbox, hs);
    // every reverse step adds its blocks' parameter terms to their partials;
    // one reduction over each box's blocks follows the sweep
    if (e == hipSuccess)
        e = launch_fill_f64(a.partials, 0.0, int64_t(s->d.nblk) * kMaxParts * kPartialStride, hs);
    double *const lo_x[3] = {a.lo, a.lo + nt, a.lo + 2 * nt};
    double *const lo_v[3] = {a.lo + 3 * nt, a.lo + 4 * nt, a.lo + 5 * nt};
    Pos wa = a.wa, wb = a.wb;
    auto hvp = [&](Buffers &bl, const Pos &x, double mult, bool drift_adj) {
        if (e == hipSuccess) {
            Timed t(s, TMD_T_ADJOINT, hs);
            e = launch_hvp(s->d, bl, x, wa, a.lx, wb, mult, drift_adj, a.partials, hs);
        }
        if (drift_adj)
            std::swap(wa, wb);
    };
    // the system holds x_T with the list of force evaluation T
    if (e == hipSuccess)
        e = launch_gather(s->d, lam_x, b.orig[s->cur.o], a.lx, hs);
    if (e == hipSuccess)
        e = launch_gather(s->d, (lam_v && lam_v[0] && lam_v[1] && lam_v[2]) ? lam_v : nullptr, b.orig[s->cur.o], wa,
                          hs);
    hvp(b, b.pos(s->cur.x), 1.0, true);
    if (e == hipSuccess)
        e = launch_unload(s->d, a.lx.x, a.lx.y, a.lx.z, b.orig[s->cur.o], lo_x, hs);
    if (e == hipSuccess)
        e = launch_unload(s->d, wa.x, wa.y, wa.z, b.orig[s->cur.o], lo_v, hs);
    for (int32_t m = nseg - 1; m >= 0 && e == hipSuccess; --m) {
        const int32_t k_lo = m * R, k_hi = std::min((m + 1) * R, T) - 1;
        // the interval's list, atom order and first positions, as the
        // forward pass built them; its later positions are in the store
        AdjList l{};
        carve_adj_list(s->dmax, a.lists + size_t(m) * a.list_bytes, &l);
        Buffers bl = b;
        bl.nbr = l.nbr;
        bl.nbr_count = l.cnt;
        bl.hood_tab = l.hood;
        const size_t np = size_t(s->d.ntp);
        auto traj = [&](int32_t j) {
            if (j == 0)
                return l.x;
            double *t = a.traj + size_t(k_lo + j) * 3 * np;
            return Pos{t, t + np, t + 2 * np};
        };
        if (e == hipSuccess)
            e = launch_gather(s->d, lo_x, l.orig, a.lx, hs);
        if (e == hipSuccess)
            e = launch_gather(s->d, lo_v, l.orig, wa, hs);
        for (int32_t k = k_hi; k >= k_lo; --k)
            hvp(bl, traj(k - k_lo), k == 0 ? 1.0 : 2.0, k > 0);
        double *const *ox = (m == 0) ? grad_x0 : lo_x;
        if (e == hipSuccess)
            e = launch_unload(s->d, a.lx.x, a.lx.y, a.lx.z, l.orig, ox, hs);
        if (m > 0) {
            if (e == hipSuccess)
                e = launch_unload(s->d, wa.x, wa.y, wa.z, l.orig, lo_v, hs);
        } else if (grad_v0 && grad_v0[0] && grad_v0[1] && grad_v0[2]) {
            if (e == hipSuccess)
                e = launch_unload(s->d, wa.x, wa.y, wa.z, l.orig, grad_v0, hs);
        }
    }
    if (e == hipSuccess)
        e = launch_grad_reduce(s->d, b, a.partials, 1.0, a.acc, hs);
    if (e == hipSuccess && (grad_eps || grad_sigma))
        e = launch_split_pairs(a.acc, s->d.nbox, grad_eps, grad_sigma, hs);
    // leave the system in the recorded final state
    if (e == hipSuccess) {
        const double *c = a.ckpt + size_t(nseg) * 6 * nt;
        const double *const po[3] = {c, c + nt, c + 2 * nt};
        const double *const vo[3] = {c + 3 * nt, c + 4 * nt, c + 5 * nt};
        e = launch_load_state(s->d, po, vo, b, Cursor{}, hs);
    }
    if (e != hipSuccess)
        return hip_fail(s, e, "adjoint_backward");
    s->cur = Cursor{};
    s->list_valid = s->force_valid = false;
    s->step = s->adj.step0 + T;
    s->adj.gen = ++s->gen;  // a second backward over the same run stays valid
    return TMD_OK;
}

tmd_status tmd_set_timing(tmd_system *s, int32_t enable) {
    if (!s)
        return TMD_EINVAL;
    s->timing = enable != 0;
    return TMD_OK;
}

tmd_status tmd_set_graphs(tmd_system *s, int32_t enable) {
    if (!s)
        return TMD_EINVAL;
    s->graphs = enable != 0;
    if (!s->graphs)
        drop_segs(s);
    return TMD_OK;
}

tmd_status tmd_get_timing(tmd_system *s, double *ms, int64_t *launches) {
    if (!s || !ms || !launches)
        return TMD_EINVAL;
    for (auto &ev : s->pending) {
        hipError_t e = hipEventSynchronize(ev.b);
        float t = 0.0f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&t, ev.a, ev.b);
        if (e != hipSuccess)
            return hip_fail(s, e, "get_timing");
        s->t_ms[ev.cls] += t;
        s->t_n[ev.cls] += ev.n;
        s->pool.push_back(ev.a);
        s->pool.push_back(ev.b);
    }
    s->pending.clear();
    for (int k = 0; k < TMD_T_COUNT; ++k) {
        ms[k] = s->t_ms[k];
        launches[k] = s->t_n[k];
        s->t_ms[k] = 0.0;
        s->t_n[k] = 0;
    }
    return TMD_OK;
}

tmd_status tmd_compute_forces_static(const tmd_params *p, int64_t n_atoms, double L, const double *const pos[3],
                                     double *const f[3], double *ev, int32_t *device_status, tmd_stream stream) {
    if (!p || !pos || !pos[0] || !pos[1] || !pos[2])
        return TMD_EINVAL;
    // the schedule tmd_create picks, on the stack
    Box B;
    tmd_status st = make_box(*p, n_atoms, L, 0, B);
    if (st != TMD_OK)
        return st;
    Dims d{};
    d.nt = int32_t(n_atoms);
    d.ntp = round_up(d.nt + 1, 256);
    d.nbox = 1;
    d.maxnb = p->max_neighbors;
    d.nchunk = (d.maxnb + 3) / 4 + 1;
    d.model = p->model;
    if (!layout_dims(&B, 1, default_edge(&B, 1), d))
        return TMD_EINVAL;
    if (carve(d, nullptr, nullptr) > size_t(TMD_STATIC_SCRATCH_BYTES))
        return TMD_EWORKSPACE;
    StaticDevice sd;
    if ((st = static_device(sd)) != TMD_OK)
        return st;
    fit_cap(d, sd.max_lds);
    Buffers b{};
    carve(d, static_cast<char *>(sd.ptr), &b);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    Cursor cur;
    hipError_t e = launch_store_box(b.boxes, B, hs);
    if (e == hipSuccess)
        e = launch_fill_i32(b.blk_box, 0, d.nblk, hs);
    if (e == hipSuccess)
        e = launch_fill_i32(b.atom_box, 0, d.ntp, hs);
    if (e == hipSuccess)
        e = launch_fill_i32(b.err, 0, 16, hs);
    if (e == hipSuccess)
        e = launch_load_state(d, pos, nullptr, b, cur, hs);
    if (e == hipSuccess)
        e = launch_bin(d, b, cur, false, hs);
    cur.x = 1 - cur.x;
    cur.o = 1 - cur.o;
    cur.v = 1 - cur.v;
    if (e == hipSuccess)
        e = launch_build(d, b, cur, hs);
    if (e == hipSuccess)
        e = launch_force(d, b, cur, 0, ev != nullptr, hs);
    if (e == hipSuccess && ev)
        e = launch_reduce(d, b, ev, 2, hs);
    if (e == hipSuccess && f && (f[0] || f[1] || f[2]))
        e = launch_unload(d, b.fx, b.fy, b.fz, b.orig[cur.o], f, hs);
    if (e == hipSuccess && device_status)
        e = launch_status_out(b.err, device_status, hs);
    return e == hipSuccess ? TMD_OK : TMD_EHIP;
}

void tmd_destroy(tmd_system *s) {
    if (!s)
        return;
    for (auto &ev : s->pending) {
        (void)hipEventSynchronize(ev.b);
        (void)hipEventDestroy(ev.a);
        (void)hipEventDestroy(ev.b);
    }
    for (hipEvent_t e : s->pool)
        (void)hipEventDestroy(e);
    drop_segs(s);
    if (s->cap_stream)
        (void)hipStreamDestroy(s->cap_stream);
    delete s;
}

}  // extern "C"

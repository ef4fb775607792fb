// Internal declarations of librbe2d: the handle, the per-system descriptor
// tables, device helpers and the kernel launchers shared by the translation
// units of the library.
//
// A handle holds n_sys >= 1 independent slabs ("systems").  A single-system
// handle is a batch of one.  Every kernel finds the system of its block (or
// wave) in small layout tables, so one launch of each kernel covers all
// systems of a batch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rbe2d.h"

namespace rbe2d {

constexpr int kBlock = 256;          // threads per block of the particle kernels
constexpr int kMaxTileThreads = 16;  // particles per thread in one structure-factor tile
constexpr int kTileMax = kBlock * kMaxTileThreads;
constexpr int kKChunk32 = 16;        // k-vectors per structure-factor block, FP32 phases
constexpr int kKChunk64 = 8;         // k-vectors per structure-factor block, FP64
constexpr int kPPad = 16;            // P is padded to a multiple of this
constexpr int kMaxFamilies = 128;    // real-space image families (order, side) per system
constexpr int kWave = 64;
constexpr int kMaxRealSplit = 5;     // real space: column groups a target's pair work may be split into
constexpr double kPi = 3.14159265358979323846;

// One family of image sources for the real-space sum, seen from the target:
// the order-l image of source j above/below the slab is at the same
// distance from r_i as the real source j is from the transformed target
// (x_i, y_i, sz * z_i + cz).  A z-force computed at the transformed target
// is multiplied by zsign.  dwt/dwb are the derivatives of the weight w
// with respect to gamma_top/gamma_bot.
struct Family {
    double sz, cz, w, zsign, dwt, dwb;
};

// Image weights and the exponents (of gamma_top, gamma_bot) of each weight,
// index l-1, for the + (above) and - (below) image of order l.
struct ImgTable {
    double gp[64], gm[64];
    int ea_p[64], eb_p[64], ea_m[64], eb_m[64];
};

// Parameters and derived constants of one system (device copy).
struct SysDesc {
    double Lx, Ly, H, Lz, V, S, alpha, rc, rc2, pref;
    double g_top, g_bot;
    double g1, cgam, dg1t, dg1b, dcgt, dcgb;   // IBC image-dipole coefficients
    double cfac;                               // 2 pi S pref / (V P)
    double scale_h;                            // 2^fh_bits (FP32 phase split)
    double hx, hy, hz, inv_hx, inv_hy, inv_hz;  // cell sizes
    double rc_lay, H_rc;                       // r_c (1 + 1e-9): layer ranges; H + r_c: image families in reach
    double inv_Lx, inv_Ly, inv_Lz;
    int ncx, ncy, ncz, reach, reach_y, nfam, M, fh_bits, cbase;
    int nmax[3], cdf_off[3];                   // sampler tables in the shared CDF array
    // fixed-point source records of the FP32 pair kernel: x and y in units
    // of period / 2^32 (so an int32 difference is the minimum image), z + zoff
    // in units of zspan / 2^32; pairs closer than `near` use FP64 geometry.
    // Isotropic frame (iso = 1): Lx = Ly and z takes the x unit too, which is
    // exact for every candidate because |dz| < Lx / 2; the pair kernel then
    // tests distances in units squared and scales only accepted pairs.
    double fxs, fys, fzs, zoff;                // scale factors 2^32 / (Lx, Ly, zspan)
    float ux, uy, uz, rc2f, near2f;            // units as floats, r_c^2, near^2
    int iso;
    float u2, rc2q, near2q;                    // iso: ux^2, r_c^2 / ux^2, near^2 / ux^2
    double ud;                                 // iso: ux in FP64
    // surface charges on the interfaces (surf = 1 when either is nonzero):
    // the sheets' uniform field Es and potential offset Cs in the slab
    // (phi_s(z) = -Es z + Cs), and the image sums of the net-charge term,
    // Gs = sum_w w, A1 = sum_w w s_w c_w, A0 = sum_w w c_w^2 over the real
    // charge and its images z_w = s_w z + c_w; each with its derivatives by
    // gamma_top, gamma_bot ([1], [2])
    double sig_top, sig_bot;
    double Es[3], Cs[3], Gs[3], A1[3], A0[3];
    int surf;
};

// Per-system scalars of the IBC and surface terms (kspace.hip: ibc_scalars)
constexpr int kScal = 20;

// Per-k record written by the reduce/assemble kernel (FP64):
//   [0..2] kx, ky, kz      [3..6] c*A (re, im), c*B (re, im)
//   [7] e_l = c Re(rho conj(rho^M))   [8..9] d e_l / d gamma_{top,bot}
//   [10..12] nx, ny, nz (as doubles)  [13..14] rho (re, im)  [15] kx^2 + ky^2
//   [16..19] polar form |cA|, arg cA / 2 pi, |cB|, arg cB / 2 pi
constexpr int kKRec = 20;

// Layout of the particles of all systems in the internal arrays (device
// copies, n_sys + 1 entries each, prefix form: entry r is the start of
// system r, entry n_sys the total).
struct Layout {
    int *off = nullptr;     // caller particle offsets
    int *pbase = nullptr;   // padded k-space particle offsets (multiples of the tile)
    int *bbase = nullptr;   // pbase / kBlock: particle blocks
    int *tbase = nullptr;   // pbase / tile: structure-factor tiles
    int *sbase = nullptr;   // padded real-space offsets (multiples of a wave)
};

// HIP-event timing of kernel classes (rbe2d_profile_enable / _read)
struct Profiler {
    int n = 0;                               // event pairs per class
    uint32_t mask = ~0u;                     // classes timed
    std::vector<hipEvent_t> ev[RBE2D_PROF_SLOTS][2];
    int used[RBE2D_PROF_SLOTS] = {};
};

struct Workspace {
    SysDesc *sys = nullptr;
    ImgTable *img = nullptr;
    Family *fam = nullptr;      // kMaxFamilies per system
    double *cdf = nullptr;      // sampler tables of all systems
    Layout lay;
    // particles (k-space arrays padded per system to whole tiles)
    float4 *p32 = nullptr;      // 2 per particle: (fxh, fxl, fyh, fyl), (fzh, fzl, q, 0)
    double4 *p64 = nullptr;     // 1 per particle: (fx, fy, fz, q)
    double *bpart = nullptr;    // per particle block: sum q z, sum q, sum q^2, sum q z^2
    double *scal = nullptr;     // kScal scalars per system, see kspace.hip
    // k-space (P_pad k-vectors per system)
    int32_t *kset = nullptr;    // n_sys x P x 3
    float4 *kn32 = nullptr;     // per k: (nx, ny, nz, 0) as floats
    double4 *kn64 = nullptr;    // per k: (nx, ny, nz, 0) as doubles
    void *sfpart = nullptr;     // structure-factor partials [tile][P_pad][4] (FP64)
    double *krec = nullptr;     // per-k records, kKRec doubles each (n_sys x P)
    float4 *kf32 = nullptr;     // per k: (kx, ky, kz, kx^2 + ky^2), (cAr, cAi, cBr, cBi),
                                // (|cA|, arg cA / 2 pi, |cB|, arg cB / 2 pi)
    double *fpart = nullptr;    // force-pass partials [ksplit][blocks * kBlock][4]
    // real space
    int *cell = nullptr, *slot = nullptr, *count = nullptr, *start = nullptr;
    int2 *tmp = nullptr;        // unordered cell lists: (caller index, global cell)
    int *scanbuf = nullptr;     // per-scan-block totals of the cell counts
    double4 *sorted = nullptr;  // (x - x0(cell), y, z, q) in cell order, padded per system
    uint4 *src16 = nullptr;     // the same particles as fixed-point (x, y, z) and FP32 q (FP32 kernel)
    int *sidx = nullptr;        // caller index of sorted particle
    int *scell = nullptr;       // local cell of sorted particle
    double4 *freal = nullptr;   // per caller particle: F_real (x, y, z), phi_real
    double2 *dgreal = nullptr;  // per caller particle: d phi_real / d gamma_{top,bot}
    double *rpart = nullptr;    // per real-space wave: sum q phi, sum q dphi/dg_top, .../dg_bot
    // partial real-space outputs when the pair work of each target is split
    // over several blocks (small N): [split][split_cap] / [split][waves]
    double4 *freal_s = nullptr;
    double2 *dgreal_s = nullptr;
    double *rpart_s = nullptr;
    double *spart = nullptr;    // per real-space wave: short-range pair and wall energies
    int *err = nullptr;         // device error word
    long long *step = nullptr;  // device MD step counter (graph replays)
};

// MD extras in the form the kernels use (from rbe2d_md_params).
struct MdExtra {
    double c1, c2;                 // BAOAB O-step: v = c1 v + c2 xi
    double sig2, eps, rc2;         // ion-ion WCA: sigma^2, eps, (2^(1/6) sigma)^2
    double sigw2, epsw, hcut;      // wall WCA: sigma_w^2, eps_w, 2^(1/6) sigma_w
    double margin;                 // reflecting walls of the integrator
    bool short_on() const { return eps != 0.0 || epsw != 0.0; }
};
constexpr uint64_t kThermoStream = 1ull << 63;   // stream ids of the thermostat noise

// Host copy of one system's setup.
struct SysHost {
    rbe2d_params p{};
    SysDesc d{};
    ImgTable img{};
    std::vector<Family> fam;
    std::vector<std::vector<double>> cdf;   // per axis
};

}  // namespace rbe2d

struct rbe2d_ctx {
    int n_sys = 1;
    bool batch = false;
    int precision = RBE2D_PREC_FP64;
    int P = 0, P_pad = 0;
    int device = 0;
    std::vector<rbe2d::SysHost> sys;
    int64_t n_cap = 0;               // caller particles (sum of n_max)
    int64_t cap_particles = 0;       // padded k-space capacity (all systems)
    int64_t cap_sorted = 0;          // padded real-space capacity
    int total_cells = 0;
    bool iso = false;                // every system has the isotropic fixed-point frame
    int64_t split_cap = 0;           // targets per split of the partial real-space outputs
    int64_t fpart_blocks = 0;        // particle blocks' worth of force-pass partials (k-range splits)
    bool one_stream = false;         // run the k-space chain on the caller's stream too (no side stream)
    bool cells_counted = false;      // the last MD pass counted the particles per cell (next build skips it)
    bool kset_valid = false;
    // current layout (host mirror); a layout is uploaded when it changes
    std::vector<int> lay_host;       // 5 x (n_sys + 1): off, pbase, bbase, tbase, sbase
    bool lay_valid = false;
    int per = 0;                     // particles per thread of the structure-factor tiles
    int64_t n_total = 0;
    int n_blocks = 0, n_tiles = 0, n_swaves = 0;
    int *lay_stage = nullptr;        // pinned staging of layout uploads
    hipEvent_t lay_ev = nullptr;
    bool lay_ev_pending = false;
    rbe2d::Workspace w;
    std::vector<void *> allocs;
    int32_t *kstage = nullptr;       // pinned staging of host k-set uploads
    hipEvent_t kev = nullptr;        // completion of the last upload from kstage
    // the k-space chain runs on a second stream beside the real-space chain
    // (default priority), forked from and joined back to the caller's stream
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr, tail_ev = nullptr;
    bool kev_pending = false;
    // launch parameters: tuned for one particle layout by rbe2d_autotune, else
    // heuristic; force_* override both while the tuner times candidates
    struct Tuning {
        std::vector<int64_t> counts;   // per-system particle counts the values were tuned for
        int per = 0, ksplit = 0, rsplit = 0;
    } tune;
    bool tuned_now = false;          // the current layout is the tuned one
    int force_per = 0, force_ksplit = 0, force_rsplit = 0;
    // cached graph of one MD step
    hipGraphExec_t md_exec = nullptr;
    hipGraph_t md_graph = nullptr;
    std::vector<uint64_t> md_key;    // arguments and layout the graph was captured for
    // every call that changes the workspaces bumps `calls`; rbe2d_energy
    // records the state it left, which rbe2d_energy_backward reuses when
    // nothing ran in between on the same inputs
    uint64_t calls = 0;
    struct {
        uint64_t at = ~0ull;
        const double *pos = nullptr, *q = nullptr;
        int64_t n = -1;
    } fwd;
    rbe2d::Profiler prof;
    std::string err;
};

namespace rbe2d {

// kernel launchers (return hipSuccess or the launch error); all systems at once
// k-vector table, particle records and IBC block sums; with scalars, also
// the IBC scalars (else the assembly launch computes them)
hipError_t launch_prep(rbe2d_ctx *h, const double *pos, const double *q, hipStream_t s, bool scalars = true);
// structure factors and per-k assembly; with_scalars: the assembly launch
// also computes the IBC scalars (otherwise the prep launch does)
// want_dg: also the per-k gamma derivatives of the energy (for dE/dgamma)
hipError_t launch_kcoef_sf(rbe2d_ctx *h, hipStream_t s, bool with_scalars = false, bool want_dg = false);
// k-vector tables of the current k-set (kn32, kn64)
void launch_ktable(rbe2d_ctx *h, hipStream_t s);
hipError_t launch_kforce(rbe2d_ctx *h, const double *pos, const double *q, double *F, double *dEdq,
                         uint32_t flags, bool accumulate, bool want_pot, bool add_real, const double *gE,
                         hipStream_t s, double *var = nullptr);
hipError_t launch_real(rbe2d_ctx *h, const double *pos, const double *q, bool want_dg, hipStream_t s);
hipError_t launch_cells(rbe2d_ctx *h, const double *pos, const double *q, hipStream_t s);
hipError_t launch_pairs(rbe2d_ctx *h, bool want_dg, hipStream_t s);
hipError_t launch_add_real(rbe2d_ctx *h, double *F, double *vel, double half_dt, hipStream_t s);
// short-range forces added to F, or with into_real to the pair kernel's
// per-particle output (then folded into F with the real-space forces)
hipError_t launch_short(rbe2d_ctx *h, const MdExtra &mx, double *F, double *energy, hipStream_t s,
                        bool into_real = false);
hipError_t launch_md_kick_drift_langevin(rbe2d_ctx *h, double *pos, double *vel, const double *F, double dt,
                                         const MdExtra &mx, uint64_t seed, uint64_t stream_base,
                                         const long long *dev_step, hipStream_t s);
hipError_t launch_energy(rbe2d_ctx *h, double *energy, uint32_t flags, const double *gE, double *dEdgamma,
                         hipStream_t s);
hipError_t launch_sample(rbe2d_ctx *h, uint64_t seed, uint64_t stream_id, const long long *dev_step,
                         hipStream_t s);
hipError_t launch_md_kick(rbe2d_ctx *h, double *vel, const double *F, double dt, hipStream_t s);
// MD update fused with the k-space particle preparation (the k-vector table
// follows each k-draw and the IBC scalars come with the assembly, so the
// side stream starts with the structure factors): the opening half kick and drift
// with F (with_real false), or, between two velocity-Verlet steps, the
// closing and next opening half kicks with F plus the real-space part and
// the drift (with_real true)
hipError_t launch_prep_md(rbe2d_ctx *h, double *pos, double *vel, const double *F, const double *q, double dt,
                          double zlo, double zhi_from_top, bool with_real, hipStream_t s);
hipError_t launch_set_step(rbe2d_ctx *h, long long value, hipStream_t s);
hipError_t launch_step_inc(rbe2d_ctx *h, hipStream_t s);
hipError_t launch_fill(void *p, int64_t nbytes_multiple_of_4, hipStream_t s);

int choose_tile(int64_t N_total, int n_kchunks);
int choose_ksplit(int64_t n_blocks, int P);

// bracket a launch of kernel class `slot` with profiling events (no-op when off)
inline void prof_begin(rbe2d_ctx *h, int slot, hipStream_t s) {
    Profiler &p = h->prof;
    if (p.n > 0 && ((p.mask >> slot) & 1u) && p.used[slot] < p.n)
        (void)hipEventRecord(p.ev[slot][0][p.used[slot]], s);
}
inline void prof_end(rbe2d_ctx *h, int slot, hipStream_t s) {
    Profiler &p = h->prof;
    if (p.n > 0 && ((p.mask >> slot) & 1u) && p.used[slot] < p.n)
        (void)hipEventRecord(p.ev[slot][1][p.used[slot]++], s);
}

// Local cell of a particle: z-layer slowest, then x, then y (rows along y
// are contiguous); xw, yw receive the wrapped lateral position.
__device__ __forceinline__ int cell_of(double x, double y, double z, const SysDesc &d, double *xw, double *yw) {
    double fx = x / d.Lx; fx -= floor(fx);
    double fy = y / d.Ly; fy -= floor(fy);
    *xw = fx * d.Lx;
    *yw = fy * d.Ly;
    const int cx = min(d.ncx - 1, max(0, (int)(*xw / d.hx)));
    const int cy = min(d.ncy - 1, max(0, (int)(*yw / d.hy)));
    const int cz = min(d.ncz - 1, max(0, (int)(z / d.hz)));   // z outside (0,H) is flagged by prep
    return (cz * d.ncx + cx) * d.ncy + cy;
}

// Largest r in [0, n) with a[r] <= x, for a nondecreasing prefix array a[0..n].
__host__ __device__ inline int find_sys(const int *a, int n, int x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// SplitMix64 stream used by the host and device k-samplers.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
__host__ __device__ inline uint64_t stream_key(uint64_t seed, uint64_t stream_id) {
    uint64_t base = mix64(seed);
    return mix64(base + (stream_id + 1) * kGolden);
}
__host__ __device__ inline double uniform01(uint64_t key, uint64_t counter) {
    return (double)(mix64(key + (counter + 1) * kGolden) >> 11) * (1.0 / 9007199254740992.0);
}
__host__ __device__ inline int draw_axis(const double *cdf, int nmax, double u) {
    int lo = 0, hi = 2 * nmax;   // smallest m with u < cdf[m]
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (u < cdf[mid]) hi = mid; else lo = mid + 1;
    }
    return lo - nmax;
}

}  // namespace rbe2d

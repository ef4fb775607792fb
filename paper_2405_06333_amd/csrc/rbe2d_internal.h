// Internal declarations of librbe2d: the handle, device helpers and the
// kernel launchers shared by the translation units of the library.
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
constexpr int kMaxFamilies = 128;    // real-space image families (order, side)
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

// Per-k record written by the reduce/assemble kernel (FP64):
//   [0..2] kx, ky, kz      [3..6] c*A (re, im), c*B (re, im)
//   [7] e_l = c Re(rho conj(rho^M))   [8..9] d e_l / d gamma_{top,bot}
//   [10..12] nx, ny, nz (as doubles)  [13..15] unused
constexpr int kKRec = 16;

// HIP-event timing of kernel classes (rbe2d_profile_enable / _read)
struct Profiler {
    int n = 0;                               // event pairs per class
    std::vector<hipEvent_t> ev[RBE2D_PROF_SLOTS][2];
    int used[RBE2D_PROF_SLOTS] = {};
};

struct Workspace {
    // particles (padded to a multiple of kTileMax)
    float4 *p32 = nullptr;      // 2 per particle: (fxh, fxl, fyh, fyl), (fzh, fzl, q, 0)
    double4 *p64 = nullptr;     // 1 per particle: (fx, fy, fz, q)
    double *bpart = nullptr;    // per prep block: sum q z, sum q, sum q^2, 0
    double *scal = nullptr;     // scalars, see kspace.hip
    // k-space
    float4 *kn32 = nullptr;     // per k: (nx, ny, nz, 0) as floats
    double4 *kn64 = nullptr;    // per k: (nx, ny, nz, 0) as doubles
    void *sfpart = nullptr;     // structure-factor partials [tile][P_pad][4] (float or double)
    double *krec = nullptr;     // per-k records, kKRec doubles each
    float4 *kf32 = nullptr;     // per k: (kx, ky, kz, 0), (cAr, cAi, cBr, cBi)
    double *fpart = nullptr;    // force-pass partials [ksplit][N][4]
    // real space
    int *cell = nullptr, *slot = nullptr, *count = nullptr, *start = nullptr, *tmp = nullptr;
    int *scanbuf = nullptr;     // per-scan-block totals of the cell counts
    double4 *sorted = nullptr;  // (x, y, z, q) in cell order, x relative to the cell's x edge
    int *sidx = nullptr;        // original index of sorted particle
    int *scell = nullptr;       // cell of sorted particle
    double4 *freal = nullptr;   // per original particle: F_real (x, y, z), phi_real
    double2 *dgreal = nullptr;  // per original particle: d phi_real / d gamma_{top,bot}
    double *rpart = nullptr;    // per real-space block: sum q phi, sum q dphi/dg_top, .../dg_bot
    Family *fam = nullptr;      // image families (device copy)
    ImgTable *img = nullptr;    // image weights (device copy)
    int *err = nullptr;         // device error word
    int32_t *kset = nullptr;    // P x 3
    double *cdf[3] = {nullptr, nullptr, nullptr};
};

}  // namespace rbe2d

struct rbe2d_ctx {
    rbe2d_params p{};
    double Lz = 0, V = 0, S = 0, pref = 1;
    int device = 0;
    int M = 0, P = 0, P_pad = 0;
    std::vector<double> gp, gm;      // image weights, index l-1
    double g1 = 1.0;                 // dw/dz = 1 + sum_l (-1)^l (g+ + g-)
    double cgam = 0.0;               // sum_l (2 ceil(l/2) H g+ - 2 floor(l/2) H g-)
    double dg1[2] = {0, 0}, dcgam[2] = {0, 0};   // their gamma derivatives
    int nmax[3] = {0, 0, 0};
    int fh_bits = 12;                // fraction bits of the FP32 phase split
    std::vector<std::vector<double>> cdf_host;
    bool kset_valid = false;
    int64_t n_cap = 0;               // padded particle capacity
    int n_tiles_cap = 0;
    // cell grid
    int ncx = 1, ncy = 1, ncz = 1, ncells = 1;
    int reach = 2;                   // neighbour columns on each side; cells >= r_c / reach
    int round_min = 40;              // real space: drain pair queues while >= this many lanes hold work
    double hx = 0, hy = 0, hz = 0;
    std::vector<rbe2d::Family> fam;
    rbe2d::Workspace w;
    std::vector<void *> allocs;
    int32_t *kstage = nullptr;       // pinned staging of host k-set uploads
    hipEvent_t kev = nullptr;        // completion of the last upload from kstage
    bool kev_pending = false;
    rbe2d::Profiler prof;
    std::string err;
};

namespace rbe2d {

// kernel launchers (return hipSuccess or the launch error)
hipError_t launch_prep(rbe2d_ctx *h, int64_t N, int64_t N_pad, const double *pos, const double *q,
                       hipStream_t s);
hipError_t launch_kcoef_sf(rbe2d_ctx *h, int64_t N_pad, int tile, hipStream_t s);
hipError_t launch_kforce(rbe2d_ctx *h, int64_t N, const double *pos, const double *q, double *F,
                         double *dEdq, uint32_t flags, bool accumulate, bool want_pot,
                         bool add_real, const double *gE, hipStream_t s);
hipError_t launch_real(rbe2d_ctx *h, int64_t N, const double *pos, const double *q, bool want_dg,
                       hipStream_t s);
hipError_t launch_energy(rbe2d_ctx *h, int64_t N, double *energy, uint32_t flags,
                         const double *gE, double *dEdgamma, hipStream_t s);
hipError_t launch_sample(rbe2d_ctx *h, uint64_t seed, uint64_t stream_id, hipStream_t s);
hipError_t launch_md_kick_drift(rbe2d_ctx *h, int64_t N, double *pos, double *vel,
                                const double *F, double dt, double zlo, double zhi,
                                hipStream_t s);
hipError_t launch_md_kick(rbe2d_ctx *h, int64_t N, double *vel, const double *F, double dt,
                          hipStream_t s);
hipError_t launch_fill(void *p, int64_t nbytes_multiple_of_4, hipStream_t s);

// bracket a launch of kernel class `slot` with profiling events (no-op when off)
inline void prof_begin(rbe2d_ctx *h, int slot, hipStream_t s);
inline void prof_end(rbe2d_ctx *h, int slot, hipStream_t s);

int choose_tile(int64_t N, int n_kchunks);
int choose_ksplit(int64_t N, int P);

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

inline void prof_begin(rbe2d_ctx *h, int slot, hipStream_t s) {
    Profiler &p = h->prof;
    if (p.n > 0 && p.used[slot] < p.n) (void)hipEventRecord(p.ev[slot][0][p.used[slot]], s);
}
inline void prof_end(rbe2d_ctx *h, int slot, hipStream_t s) {
    Profiler &p = h->prof;
    if (p.n > 0 && p.used[slot] < p.n) (void)hipEventRecord(p.ev[slot][1][p.used[slot]++], s);
}

}  // namespace rbe2d

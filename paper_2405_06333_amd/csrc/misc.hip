// Energies, the on-device k-sampler and the velocity-Verlet integrator, for
// all systems of a handle at once.
#include "devmath.h"
#include "rbe2d_internal.h"

namespace rbe2d {

// ---------------------------------------------------------------------------
// energy components {total, real, kspace, self, ibc} per system and, in
// backward mode, gE * dE/dgamma_{top,bot}.  One block per system, fixed
// summation order.
// ---------------------------------------------------------------------------

struct EnergyArgs {
    const double *krec, *rpart, *scal;
    const SysDesc *sys;
    Layout lay;
    int P;
    int do_real, do_k, do_ibc, want_dg;
    double *energy;          // 5 per system
    const double *gE;
    double *dEdgamma;        // 2 per system
};

__global__ __launch_bounds__(kBlock) void k_energy(EnergyArgs a) {
    __shared__ double sh[kBlock / 64];
    const int r = blockIdx.x;
    const SysDesc &d = a.sys[r];
    double ek = 0.0, dkt = 0.0, dkb = 0.0, er = 0.0, drt = 0.0, drb = 0.0;
    if (a.do_k)
        for (int l = threadIdx.x; l < a.P; l += kBlock) {
            const double *rec = a.krec + ((int64_t)r * a.P + l) * kKRec;
            ek += rec[7];
            dkt += rec[8];
            dkb += rec[9];
        }
    const bool has_real = a.do_real && a.lay.off[r + 1] > a.lay.off[r];
    if (has_real)
        for (int wv = a.lay.sbase[r] / kWave + threadIdx.x; wv < a.lay.sbase[r + 1] / kWave; wv += kBlock) {
            er += a.rpart[3 * wv];
            drt += a.rpart[3 * wv + 1];
            drb += a.rpart[3 * wv + 2];
        }
    ek = block_sum(ek, sh);
    er = block_sum(er, sh);
    if (a.want_dg) {
        dkt = block_sum(dkt, sh); dkb = block_sum(dkb, sh);
        drt = block_sum(drt, sh); drb = block_sum(drb, sh);
    }
    if (threadIdx.x != 0) return;
    const double *sc = a.scal + kScal * r;
    const double tv = 2.0 * kPi / d.V * d.pref;
    const double Er = has_real ? 0.5 * er : 0.0;
    const double Ek = a.do_k ? ek : 0.0;
    const double Es = a.do_k ? -d.alpha * d.pref / sqrt(kPi) * sc[2] : 0.0;
    const double Ei = a.do_ibc ? tv * sc[0] * sc[3] + sc[14] : 0.0;   // sc[14]: surface terms (or 0)
    if (a.energy) {
        double *o = a.energy + 5 * r;
        o[0] = Er + Ek + Es + Ei;
        o[1] = Er;
        o[2] = Ek;
        o[3] = Es;
        o[4] = Ei;
    }
    if (a.want_dg && a.dEdgamma) {
        const double g = a.gE ? a.gE[r] : 1.0;
        const double ibt = a.do_ibc ? tv * sc[0] * sc[6] + sc[15] : 0.0;
        const double ibb = a.do_ibc ? tv * sc[0] * sc[7] + sc[16] : 0.0;
        a.dEdgamma[2 * r] = g * ((has_real ? 0.5 * drt : 0.0) + (a.do_k ? dkt : 0.0) + ibt);
        a.dEdgamma[2 * r + 1] = g * ((has_real ? 0.5 * drb : 0.0) + (a.do_k ? dkb : 0.0) + ibb);
    }
}

hipError_t launch_energy(rbe2d_ctx *h, double *energy, uint32_t flags, const double *gE, double *dEdgamma,
                         hipStream_t s) {
    EnergyArgs a;
    a.krec = h->w.krec; a.rpart = h->w.rpart; a.scal = h->w.scal; a.sys = h->w.sys; a.lay = h->w.lay;
    a.P = h->P;
    a.do_real = (flags & RBE2D_REAL) != 0;
    a.do_k = (flags & RBE2D_KSPACE) != 0;
    a.do_ibc = (flags & RBE2D_IBC) != 0;
    a.want_dg = dEdgamma != nullptr;
    a.energy = energy; a.gE = gE; a.dEdgamma = dEdgamma;
    prof_begin(h, 6, s);
    hipLaunchKernelGGL(k_energy, dim3(h->n_sys), dim3(kBlock), 0, s, a);
    prof_end(h, 6, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// on-device k-sampler: the same draws as the host sampler in api.hip; the
// k-set of system r uses stream id (stream_base + r), where stream_base is
// the argument or, for graph replays, n_sys times a device step counter
// ---------------------------------------------------------------------------

struct SampleArgs {
    const double *cdf;
    const SysDesc *sys;
    int n_sys, P;
    uint64_t seed, stream_base;
    const long long *dev_step;   // if set: stream_base = n_sys * (*dev_step)
    int32_t *kset;
    int *err;
};

__global__ void k_sample(SampleArgs a) {
    const int kg = blockIdx.x * blockDim.x + threadIdx.x;
    if (kg >= a.n_sys * a.P) return;
    const int r = kg / a.P, l = kg - r * a.P;
    const SysDesc &d = a.sys[r];
    const uint64_t base = a.dev_step ? (uint64_t)(*a.dev_step) * (uint64_t)a.n_sys : a.stream_base;
    const uint64_t key = stream_key(a.seed, base + (uint64_t)r);
    for (int att = 0; att < 64; att++) {
        const uint64_t c = ((uint64_t)l * 64 + att) * 3;
        const int nx = draw_axis(a.cdf + d.cdf_off[0], d.nmax[0], uniform01(key, c));
        const int ny = draw_axis(a.cdf + d.cdf_off[1], d.nmax[1], uniform01(key, c + 1));
        const int nz = draw_axis(a.cdf + d.cdf_off[2], d.nmax[2], uniform01(key, c + 2));
        if (nx | ny | nz) {
            a.kset[3 * kg] = nx; a.kset[3 * kg + 1] = ny; a.kset[3 * kg + 2] = nz;
            return;
        }
    }
    a.kset[3 * kg] = 1; a.kset[3 * kg + 1] = 0; a.kset[3 * kg + 2] = 0;
    atomicOr(a.err, 2);
}

hipError_t launch_sample(rbe2d_ctx *h, uint64_t seed, uint64_t stream_id, const long long *dev_step,
                         hipStream_t s) {
    SampleArgs a;
    a.cdf = h->w.cdf; a.sys = h->w.sys; a.n_sys = h->n_sys; a.P = h->P;
    a.seed = seed; a.stream_base = stream_id; a.dev_step = dev_step;
    a.kset = h->w.kset; a.err = h->w.err;
    const int n = h->n_sys * h->P;
    prof_begin(h, 8, s);
    hipLaunchKernelGGL(k_sample, dim3((n + 63) / 64), dim3(64), 0, s, a);
    prof_end(h, 8, s);
    return hipGetLastError();
}

__global__ void k_set_step(long long *step, long long v) { *step = v; }
__global__ void k_step_inc(long long *step) { *step += 1; }

hipError_t launch_set_step(rbe2d_ctx *h, long long value, hipStream_t s) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, h->w.step, value);
    return hipGetLastError();
}
hipError_t launch_step_inc(rbe2d_ctx *h, hipStream_t s) {
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(1), 0, s, h->w.step);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// integrators with unit masses; x, y periodic, z reflected at the walls.
// The plain velocity-Verlet update is fused into the k-space preparation
// (k_prep with MD > 0); the Langevin one and the half kick are here.
// ---------------------------------------------------------------------------

// BAOAB up to the force evaluation (Langevin equation, unit masses):
// v += dt/2 F; r += dt/2 v; v = c1 v + c2 xi; r += dt/2 v; wrap / reflect.
// xi: Box-Muller normals from the SplitMix64 stream (seed, 2^63 + step n_sys
// + system), uniforms 2(3i+c) and 2(3i+c)+1 for particle i of its system.
__global__ __launch_bounds__(kBlock) void k_kick_drift_langevin(const SysDesc *sys, Layout lay, int n_sys,
                                                                int n_total, double *pos, double *vel,
                                                                const double *F, double dt, double c1, double c2,
                                                                double margin, uint64_t seed, uint64_t stream_base,
                                                                const long long *dev_step) {
    const int g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= n_total) return;
    const int r = find_sys(lay.off, n_sys, g);
    const SysDesc &d = sys[r];
    const int64_t i = g;
    const uint64_t local = (uint64_t)(g - lay.off[r]);
    const uint64_t base = dev_step ? (uint64_t)(*dev_step) * (uint64_t)n_sys : stream_base;
    const uint64_t key = stream_key(seed, kThermoStream + base + (uint64_t)r);
    const double h = 0.5 * dt;
    double v[3], x[3];
    for (int c = 0; c < 3; c++) {
        v[c] = fma(h, F[3 * i + c], vel[3 * i + c]);
        x[c] = fma(h, v[c], pos[3 * i + c]);
        const uint64_t k = 3 * local + c;
        const double u1 = uniform01(key, 2 * k), u2 = uniform01(key, 2 * k + 1);
        const double xi = sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * kPi * u2);
        v[c] = fma(c1, v[c], c2 * xi);
        x[c] = fma(h, v[c], x[c]);
    }
    x[0] -= d.Lx * floor(x[0] / d.Lx);
    x[1] -= d.Ly * floor(x[1] / d.Ly);
    const double zlo = margin, zhi = d.H - margin;
    const double W = zhi - zlo;
    const double u = x[2] - zlo;
    const double m = floor(u / W);
    const double rem = u - m * W;
    const bool odd = fmod(fabs(m), 2.0) == 1.0;
    x[2] = odd ? zhi - rem : zlo + rem;
    if (odd) v[2] = -v[2];
    x[2] = fmin(fmax(x[2], zlo), zhi);
    for (int c = 0; c < 3; c++) {
        vel[3 * i + c] = v[c];
        pos[3 * i + c] = x[c];
    }
}

hipError_t launch_md_kick_drift_langevin(rbe2d_ctx *h, double *pos, double *vel, const double *F, double dt,
                                         const MdExtra &mx, uint64_t seed, uint64_t stream_base,
                                         const long long *dev_step, hipStream_t s) {
    if (h->n_total == 0) return hipSuccess;
    prof_begin(h, 7, s);
    hipLaunchKernelGGL(k_kick_drift_langevin, dim3((unsigned)((h->n_total + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, h->w.sys, h->w.lay, h->n_sys, (int)h->n_total, pos, vel, F, dt, mx.c1, mx.c2, mx.margin,
                       seed, stream_base, dev_step);
    prof_end(h, 7, s);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_kick(int64_t n3, double *vel, const double *F, double dt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n3) return;
    vel[i] = fma(0.5 * dt, F[i], vel[i]);
}

hipError_t launch_md_kick(rbe2d_ctx *h, double *vel, const double *F, double dt, hipStream_t s) {
    if (h->n_total == 0) return hipSuccess;
    const int64_t n3 = 3 * h->n_total;
    prof_begin(h, 7, s);
    hipLaunchKernelGGL(k_kick, dim3((unsigned)((n3 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n3, vel, F, dt);
    prof_end(h, 7, s);
    return hipGetLastError();
}

}  // namespace rbe2d

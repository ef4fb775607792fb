// Energies, the on-device k-sampler and the velocity-Verlet integrator.
#include "devmath.h"
#include "rbe2d_internal.h"

namespace rbe2d {

// ---------------------------------------------------------------------------
// energy components {total, real, kspace, self, ibc} and, in backward mode,
// gE * dE/dgamma_{top,bot}.  One block, fixed summation order.
// ---------------------------------------------------------------------------

struct EnergyArgs {
    const double *krec, *rpart, *scal;
    int P, n_rblocks;
    double twopi_over_V, pref, self_coef;   // self_coef = -alpha pref / sqrt(pi)
    int do_real, do_k, do_ibc, want_dg;
    double *energy;
    const double *gE;
    double *dEdgamma;
};

__global__ __launch_bounds__(kBlock) void k_energy(EnergyArgs a) {
    __shared__ double sh[kBlock / 64];
    double ek = 0.0, dkt = 0.0, dkb = 0.0, er = 0.0, drt = 0.0, drb = 0.0;
    if (a.do_k)
        for (int l = threadIdx.x; l < a.P; l += kBlock) {
            ek += a.krec[(int64_t)l * kKRec + 7];
            dkt += a.krec[(int64_t)l * kKRec + 8];
            dkb += a.krec[(int64_t)l * kKRec + 9];
        }
    if (a.do_real)
        for (int b = threadIdx.x; b < a.n_rblocks; b += kBlock) {
            er += a.rpart[3 * b];
            drt += a.rpart[3 * b + 1];
            drb += a.rpart[3 * b + 2];
        }
    ek = block_sum(ek, sh);
    er = block_sum(er, sh);
    if (a.want_dg) {
        dkt = block_sum(dkt, sh); dkb = block_sum(dkb, sh);
        drt = block_sum(drt, sh); drb = block_sum(drb, sh);
    }
    if (threadIdx.x != 0) return;
    const double Er = a.do_real ? 0.5 * er : 0.0;
    const double Ek = a.do_k ? ek : 0.0;
    const double Es = a.do_k ? a.self_coef * a.scal[2] : 0.0;
    const double Ei = a.do_ibc ? a.twopi_over_V * a.pref * a.scal[0] * a.scal[3] : 0.0;
    if (a.energy) {
        a.energy[0] = Er + Ek + Es + Ei;
        a.energy[1] = Er;
        a.energy[2] = Ek;
        a.energy[3] = Es;
        a.energy[4] = Ei;
    }
    if (a.want_dg && a.dEdgamma) {
        const double g = a.gE ? *a.gE : 1.0;
        const double ibt = a.do_ibc ? a.twopi_over_V * a.pref * a.scal[0] * a.scal[6] : 0.0;
        const double ibb = a.do_ibc ? a.twopi_over_V * a.pref * a.scal[0] * a.scal[7] : 0.0;
        a.dEdgamma[0] = g * ((a.do_real ? 0.5 * drt : 0.0) + (a.do_k ? dkt : 0.0) + ibt);
        a.dEdgamma[1] = g * ((a.do_real ? 0.5 * drb : 0.0) + (a.do_k ? dkb : 0.0) + ibb);
    }
}

hipError_t launch_energy(rbe2d_ctx *h, int64_t N, double *energy, uint32_t flags,
                         const double *gE, double *dEdgamma, hipStream_t s) {
    EnergyArgs a;
    a.krec = h->w.krec; a.rpart = h->w.rpart; a.scal = h->w.scal; a.P = h->P;
    a.n_rblocks = (int)((N + kBlock - 1) / kBlock);
    a.twopi_over_V = 2.0 * kPi / h->V; a.pref = h->pref;
    a.self_coef = -h->p.alpha * h->pref / sqrt(kPi);
    a.do_real = (flags & RBE2D_REAL) && N > 0;
    a.do_k = (flags & RBE2D_KSPACE) != 0;
    a.do_ibc = (flags & RBE2D_IBC) != 0;
    a.want_dg = dEdgamma != nullptr;
    a.energy = energy; a.gE = gE; a.dEdgamma = dEdgamma;
    prof_begin(h, 6, s);
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(kBlock), 0, s, a);
    prof_end(h, 6, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// on-device k-sampler: the same draws as the host sampler in api.hip
// ---------------------------------------------------------------------------

struct SampleArgs {
    const double *cdf0, *cdf1, *cdf2;
    int nm0, nm1, nm2, P;
    uint64_t key;
    int32_t *kset;
    int *err;
};

__global__ void k_sample(SampleArgs a) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.P) return;
    for (int att = 0; att < 64; att++) {
        const uint64_t c = ((uint64_t)l * 64 + att) * 3;
        const int nx = draw_axis(a.cdf0, a.nm0, uniform01(a.key, c));
        const int ny = draw_axis(a.cdf1, a.nm1, uniform01(a.key, c + 1));
        const int nz = draw_axis(a.cdf2, a.nm2, uniform01(a.key, c + 2));
        if (nx | ny | nz) {
            a.kset[3 * l] = nx; a.kset[3 * l + 1] = ny; a.kset[3 * l + 2] = nz;
            return;
        }
    }
    a.kset[3 * l] = 1; a.kset[3 * l + 1] = 0; a.kset[3 * l + 2] = 0;
    atomicOr(a.err, 2);
}

hipError_t launch_sample(rbe2d_ctx *h, uint64_t seed, uint64_t stream_id, hipStream_t s) {
    SampleArgs a;
    a.cdf0 = h->w.cdf[0]; a.cdf1 = h->w.cdf[1]; a.cdf2 = h->w.cdf[2];
    a.nm0 = h->nmax[0]; a.nm1 = h->nmax[1]; a.nm2 = h->nmax[2]; a.P = h->P;
    a.key = stream_key(seed, stream_id);
    a.kset = h->w.kset; a.err = h->w.err;
    prof_begin(h, 8, s);
    hipLaunchKernelGGL(k_sample, dim3((h->P + 63) / 64), dim3(64), 0, s, a);
    prof_end(h, 8, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// velocity Verlet with unit masses; x, y periodic, z reflected at zlo, zhi
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_kick_drift(int64_t N, double *pos, double *vel,
                                                       const double *F, double dt, double Lx,
                                                       double Ly, double zlo, double zhi) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    double v[3], r[3];
    for (int d = 0; d < 3; d++) {
        v[d] = fma(0.5 * dt, F[3 * i + d], vel[3 * i + d]);
        r[d] = fma(dt, v[d], pos[3 * i + d]);
    }
    r[0] -= Lx * floor(r[0] / Lx);
    r[1] -= Ly * floor(r[1] / Ly);
    // fold z into [zlo, zhi]: every crossing of a wall is a specular reflection
    const double W = zhi - zlo;
    const double u = r[2] - zlo;
    const double m = floor(u / W);
    const double rem = u - m * W;
    const bool odd = fmod(fabs(m), 2.0) == 1.0;
    r[2] = odd ? zhi - rem : zlo + rem;
    if (odd) v[2] = -v[2];
    r[2] = fmin(fmax(r[2], zlo), zhi);
    for (int d = 0; d < 3; d++) {
        vel[3 * i + d] = v[d];
        pos[3 * i + d] = r[d];
    }
}

__global__ __launch_bounds__(kBlock) void k_kick(int64_t N, double *vel, const double *F,
                                                 double dt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= 3 * N) return;
    vel[i] = fma(0.5 * dt, F[i], vel[i]);
}

hipError_t launch_md_kick_drift(rbe2d_ctx *h, int64_t N, double *pos, double *vel,
                                const double *F, double dt, double zlo, double zhi,
                                hipStream_t s) {
    if (N == 0) return hipSuccess;
    prof_begin(h, 7, s);
    hipLaunchKernelGGL(k_kick_drift, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       N, pos, vel, F, dt, h->p.Lx, h->p.Ly, zlo, zhi);
    prof_end(h, 7, s);
    return hipGetLastError();
}

hipError_t launch_md_kick(rbe2d_ctx *h, int64_t N, double *vel, const double *F, double dt,
                          hipStream_t s) {
    if (N == 0) return hipSuccess;
    prof_begin(h, 7, s);
    hipLaunchKernelGGL(k_kick, dim3((unsigned)((3 * N + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       N, vel, F, dt);
    prof_end(h, 7, s);
    return hipGetLastError();
}

}  // namespace rbe2d

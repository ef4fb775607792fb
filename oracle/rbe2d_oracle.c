/*
 * rbe2d_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, FP64 CPU reference for the random batch Ewald method for
 * dielectrically confined quasi-2D Coulomb systems (RBE2D; Gan, Gao, Liang,
 * Xu, arXiv:2405.06333).  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library: everything below is written out
 * directly from the paper's formulas with libm's sin/cos/exp/erfc.
 *
 * Geometry (Sec. 2.1, Sec. 3.1): N point charges q_i at r_i=(x_i,y_i,z_i),
 * 0 < z_i < H, periodic in x (Lx) and y (Ly); dielectric interfaces at z=0
 * (contrast gamma_bot) and z=H (contrast gamma_top).  The k-space part lives
 * on the extended periodic box Lx*Ly*Lz with Lz >= (M+1)H (Theorem 3.3).
 * Coulomb constant 1 and eps_c = 1 as in Eq. (2.1).
 *
 * Readings taken where the paper is garbled, ambiguous or silent:
 *  R1  image weights: the image of order l above the slab carries
 *      gamma_top^ceil(l/2) * gamma_bot^floor(l/2), the one below carries
 *      gamma_bot^ceil(l/2) * gamma_top^floor(l/2).  This is the physical
 *      image series and the one the closed form beta_ij(h) of Eq. (3.7)
 *      assumes; the exponents printed after Eq. (3.2) are swapped.
 *  R2  the k-space force is the gradient of rho_k * conj(rho^M_k), written
 *      out as in Eq. (3.25); the folded form printed as Eq. (3.27) has its
 *      odd/even coefficients in the wrong terms.
 *  R3  the RBE force estimator carries no extra exp(-k^2/4alpha^2) factor
 *      (importance weight S/(P k^2) only), as in Eq. (3.26); Eq. (2.20)
 *      prints a spurious Gaussian.
 *  R4  the RBE energy estimator (not printed) is the same importance-weighted
 *      sum applied to Re(rho_k conj(rho^M_k)), so that F = -grad E holds for
 *      a fixed k-set.
 *  R5  the real-space force and the IBC force (their formulas are in the
 *      missing supplement) are minus the gradients of Eq. (3.12) and of the
 *      IBC term of Theorem 3.3.
 *  R6  the real-space sum keeps pairs with distance strictly below r_c, no
 *      shift, minimum image in x and y (valid for r_c <= min(Lx,Ly)/2).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

typedef struct {
    double Lx, Ly, H, Lz;        /* Lz: extended periodic height of Theorem 3.3 */
    double g_top, g_bot;         /* dielectric contrasts, Eq. (3.1) */
    double alpha, rc;            /* Ewald splitting parameter, real-space cutoff */
    int M;                       /* image reflection order (Sec. 3.2) */
} orc_box;

/* ------------------------------------------------------------------ */
/* Image charges (Sec. 3.1, Eqs. (3.2)-(3.3), reading R1)              */
/* ------------------------------------------------------------------ */

static double ipow(double b, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; i++) r *= b;
    return r;
}

static int ceil_half(int l) { return (l + 1) / 2; }
static int floor_half(int l) { return l / 2; }

/* Exponents (a, b) of gamma_top^a * gamma_bot^b for the order-l image;
 * sign = +1 for the image above the slab, -1 for the one below. */
void orc_image_exponents(int l, int sign, int *a_top, int *b_bot)
{
    if (sign > 0) { *a_top = ceil_half(l); *b_bot = floor_half(l); }
    else          { *a_top = floor_half(l); *b_bot = ceil_half(l); }
}

void orc_image_coeffs(int M, double g_top, double g_bot, double *gp, double *gm)
{
    for (int l = 1; l <= M; l++) {
        int a, b;
        orc_image_exponents(l, +1, &a, &b);
        gp[l - 1] = ipow(g_top, a) * ipow(g_bot, b);
        orc_image_exponents(l, -1, &a, &b);
        gm[l - 1] = ipow(g_top, a) * ipow(g_bot, b);
    }
}

/* z-coordinate of the order-l image of a charge at z, Eq. (3.3). */
double orc_image_z(int l, int sign, double z, double H)
{
    double s = (l % 2 == 0) ? z : -z;
    if (sign > 0) return s + 2.0 * ceil_half(l) * H;
    return s - 2.0 * floor_half(l) * H;
}

/* ------------------------------------------------------------------ */
/* k-space (Theorem 3.3, Eqs. (3.16)-(3.18), (3.24)-(3.26))             */
/* ------------------------------------------------------------------ */

static void kvec(const orc_box *b, const int32_t *n, double *k)
{
    k[0] = 2.0 * ORC_PI * n[0] / b->Lx;
    k[1] = 2.0 * ORC_PI * n[1] / b->Ly;
    k[2] = 2.0 * ORC_PI * n[2] / b->Lz;
}

/* rho_k = sum_j q_j exp(i k.r_j) for every k of the list (Eq. (3.17)).
 * hat != 0 evaluates it at khat = (kx, ky, -kz) instead. */
void orc_rho(int64_t N, const double *pos, const double *q, const orc_box *b,
             int P, const int32_t *n, int hat, double *rho /* 2P: re,im */)
{
#pragma omp parallel for schedule(static)
    for (int l = 0; l < P; l++) {
        double k[3];
        kvec(b, n + 3 * l, k);
        if (hat) k[2] = -k[2];
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < N; j++) {
            double t = k[0] * pos[3 * j] + k[1] * pos[3 * j + 1] + k[2] * pos[3 * j + 2];
            re += q[j] * cos(t);
            im += q[j] * sin(t);
        }
        rho[2 * l] = re;
        rho[2 * l + 1] = im;
    }
}

/* rho^M_k = conj(rhobar^M_k): the structure factor of the real charges plus
 * all images up to order M, summed image by image as in Eq. (3.17). */
void orc_rhoM_explicit(int64_t N, const double *pos, const double *q, const orc_box *b,
                       int P, const int32_t *n, double *rhoM /* 2P */)
{
    double *gp = malloc(sizeof(double) * (b->M + 1));
    double *gm = malloc(sizeof(double) * (b->M + 1));
    orc_image_coeffs(b->M, b->g_top, b->g_bot, gp, gm);
#pragma omp parallel for schedule(static)
    for (int l = 0; l < P; l++) {
        double k[3];
        kvec(b, n + 3 * l, k);
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < N; j++) {
            double x = pos[3 * j], y = pos[3 * j + 1], z = pos[3 * j + 2];
            double t = k[0] * x + k[1] * y + k[2] * z;
            re += q[j] * cos(t);
            im += q[j] * sin(t);
            for (int o = 1; o <= b->M; o++) {
                double tp = k[0] * x + k[1] * y + k[2] * orc_image_z(o, +1, z, b->H);
                double tm = k[0] * x + k[1] * y + k[2] * orc_image_z(o, -1, z, b->H);
                re += q[j] * (gp[o - 1] * cos(tp) + gm[o - 1] * cos(tm));
                im += q[j] * (gp[o - 1] * sin(tp) + gm[o - 1] * sin(tm));
            }
        }
        rhoM[2 * l] = re;
        rhoM[2 * l + 1] = im;
    }
    free(gp);
    free(gm);
}

/* Recalibration coefficients of Sec. 3.4 (Eq. (3.27) and the text after it):
 *   Y_odd (kz) = sum_{l odd }[g+^(l) e^{i kz (l+1) H} + g-^(l) e^{-i kz (l-1) H}]
 *   Y_even(kz) = sum_{l even}[g+^(l) e^{i kz l H}     + g-^(l) e^{-i kz l H}]
 * so that rho^M_k = (1 + Y_even) rho_k + Y_odd rhohat_k. */
void orc_Y(const orc_box *b, int P, const int32_t *n, double *Yodd, double *Yeven)
{
    double *gp = malloc(sizeof(double) * (b->M + 1));
    double *gm = malloc(sizeof(double) * (b->M + 1));
    orc_image_coeffs(b->M, b->g_top, b->g_bot, gp, gm);
    for (int l = 0; l < P; l++) {
        double kz = 2.0 * ORC_PI * n[3 * l + 2] / b->Lz;
        double ore = 0, oim = 0, ere = 0, eim = 0;
        for (int o = 1; o <= b->M; o++) {
            if (o % 2 == 1) {
                double tp = kz * (o + 1) * b->H, tm = -kz * (o - 1) * b->H;
                ore += gp[o - 1] * cos(tp) + gm[o - 1] * cos(tm);
                oim += gp[o - 1] * sin(tp) + gm[o - 1] * sin(tm);
            } else {
                double tp = kz * o * b->H, tm = -kz * o * b->H;
                ere += gp[o - 1] * cos(tp) + gm[o - 1] * cos(tm);
                eim += gp[o - 1] * sin(tp) + gm[o - 1] * sin(tm);
            }
        }
        Yodd[2 * l] = ore; Yodd[2 * l + 1] = oim;
        Yeven[2 * l] = ere; Yeven[2 * l + 1] = eim;
    }
    free(gp);
    free(gm);
}

/*
 * k-space energy, forces and potentials for a list of P wave vectors with
 * per-k weights c[l]:
 *   E_k  = sum_l c_l Re(rho_l conj(rho^M_l))                        (R4)
 *   F_i  = -sum_l c_l grad_i Re(rho_l conj(rho^M_l))                 (Eq. (3.25), R2)
 *   phi_i = dE_k/dq_i
 * With c_l = (2 pi / V) exp(-k^2/4a^2)/k^2 over all k != 0 this is the
 * first term of Eq. (3.16); with c_l = 2 pi S / (V P k_l^2) over a sampled
 * k-set it is the RBE estimator of Eq. (3.26).
 *
 * explicit_images != 0: rho^M from Eq. (3.17) image by image and the
 * gradient from Eq. (3.25) image by image (O(P N M), the plain definition).
 * explicit_images == 0: both through Y_odd/Y_even (Sec. 3.4, O(P (N+M))).
 *
 * Outputs are written for the n_t target indices tgt[] (tgt == NULL: all
 * particles, n_t ignored).  F (n_t x 3) and phi (n_t) may be NULL.
 * rho_out (2P), rhohat_out (2P), rhoM_out (2P) may be NULL.
 */
void orc_kspace(int64_t N, const double *pos, const double *q, const orc_box *b,
                int P, const int32_t *n, const double *c, int explicit_images,
                int64_t n_t, const int64_t *tgt,
                double *E_k, double *F, double *phi,
                double *rho_out, double *rhohat_out, double *rhoM_out)
{
    double *rho = malloc(sizeof(double) * 2 * P);
    double *rhohat = malloc(sizeof(double) * 2 * P);
    double *rhoM = malloc(sizeof(double) * 2 * P);
    double *Yo = malloc(sizeof(double) * 2 * P);
    double *Ye = malloc(sizeof(double) * 2 * P);
    double *gp = malloc(sizeof(double) * (b->M + 1));
    double *gm = malloc(sizeof(double) * (b->M + 1));
    orc_image_coeffs(b->M, b->g_top, b->g_bot, gp, gm);

    orc_rho(N, pos, q, b, P, n, 0, rho);
    orc_rho(N, pos, q, b, P, n, 1, rhohat);
    orc_Y(b, P, n, Yo, Ye);
    if (explicit_images) {
        orc_rhoM_explicit(N, pos, q, b, P, n, rhoM);
    } else {
        for (int l = 0; l < P; l++) {
            /* (1 + Y_even) rho + Y_odd rhohat */
            double ar = 1.0 + Ye[2 * l], ai = Ye[2 * l + 1];
            double r = rho[2 * l], s = rho[2 * l + 1];
            double hr = rhohat[2 * l], hs = rhohat[2 * l + 1];
            rhoM[2 * l] = ar * r - ai * s + Yo[2 * l] * hr - Yo[2 * l + 1] * hs;
            rhoM[2 * l + 1] = ar * s + ai * r + Yo[2 * l] * hs + Yo[2 * l + 1] * hr;
        }
    }

    if (E_k) {
        double e = 0.0;
        for (int l = 0; l < P; l++)
            e += c[l] * (rho[2 * l] * rhoM[2 * l] + rho[2 * l + 1] * rhoM[2 * l + 1]);
        *E_k = e;
    }

    int64_t nt = tgt ? n_t : N;
    if (F || phi) {
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < nt; t++) {
            int64_t i = tgt ? tgt[t] : t;
            double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
            double fx = 0, fy = 0, fz = 0, p = 0;
            for (int l = 0; l < P; l++) {
                double k[3];
                kvec(b, n + 3 * l, k);
                double r = rho[2 * l], s = rho[2 * l + 1];
                /* Eq. (3.25): grad_i [rho rhobar^M] / q_i =
                 *   k    Im[ e^{-ik.r_i}(rho + rho^M) + sum_{l even} (g+ e^{-ik.r_i+} + g- e^{-ik.r_i-}) rho ]
                 *   khat Im[ sum_{l odd} (g+ e^{-ik.r_i+} + g- e^{-ik.r_i-}) rho ]
                 * and the same brackets with Re give dE/dq_i. */
                double u_re, u_im;        /* coefficient multiplying k    */
                double v_re, v_im;        /* coefficient multiplying khat */
                double t0 = k[0] * x + k[1] * y + k[2] * z;
                double er = cos(t0), ei = -sin(t0);        /* e^{-ik.r_i} */
                double sr = r + rhoM[2 * l], si = s + rhoM[2 * l + 1];
                u_re = er * sr - ei * si;
                u_im = er * si + ei * sr;
                v_re = 0.0; v_im = 0.0;
                if (explicit_images) {
                    for (int o = 1; o <= b->M; o++) {
                        double tp = k[0] * x + k[1] * y + k[2] * orc_image_z(o, +1, z, b->H);
                        double tm = k[0] * x + k[1] * y + k[2] * orc_image_z(o, -1, z, b->H);
                        /* (g+ e^{-i tp} + g- e^{-i tm}) * rho */
                        double wr = gp[o - 1] * cos(tp) + gm[o - 1] * cos(tm);
                        double wi = -gp[o - 1] * sin(tp) - gm[o - 1] * sin(tm);
                        double pr = wr * r - wi * s, pi_ = wr * s + wi * r;
                        if (o % 2 == 0) { u_re += pr; u_im += pi_; }
                        else            { v_re += pr; v_im += pi_; }
                    }
                } else {
                    /* even images: e^{-ik.r_i} conj(Y_even) rho ; odd: e^{-ikhat.r_i} conj(Y_odd) rho */
                    double yr = Ye[2 * l], yi = -Ye[2 * l + 1];
                    double pr = yr * r - yi * s, pi_ = yr * s + yi * r;
                    u_re += er * pr - ei * pi_;
                    u_im += er * pi_ + ei * pr;
                    double th = k[0] * x + k[1] * y - k[2] * z;
                    double hr = cos(th), hi = -sin(th);     /* e^{-ikhat.r_i} */
                    double or_ = Yo[2 * l], oi = -Yo[2 * l + 1];
                    double qr = or_ * r - oi * s, qi = or_ * s + oi * r;
                    v_re = hr * qr - hi * qi;
                    v_im = hr * qi + hi * qr;
                }
                fx -= c[l] * (k[0] * u_im + k[0] * v_im);
                fy -= c[l] * (k[1] * u_im + k[1] * v_im);
                fz -= c[l] * (k[2] * u_im - k[2] * v_im);
                p += c[l] * (u_re + v_re);
            }
            if (F) {
                F[3 * t] = q[i] * fx;
                F[3 * t + 1] = q[i] * fy;
                F[3 * t + 2] = q[i] * fz;
            }
            if (phi) phi[t] = p;
        }
    }
    if (rho_out) memcpy(rho_out, rho, sizeof(double) * 2 * P);
    if (rhohat_out) memcpy(rhohat_out, rhohat, sizeof(double) * 2 * P);
    if (rhoM_out) memcpy(rhoM_out, rhoM, sizeof(double) * 2 * P);
    free(rho); free(rhohat); free(rhoM); free(Yo); free(Ye); free(gp); free(gm);
}

/*
 * Derivative of E_k with respect to gamma_top (which = 0) or gamma_bot
 * (which = 1) at fixed positions and k-set: the weights g+-^(l) enter only
 * through rho^M (Eq. (3.17)), so
 *   dE_k/dgamma = sum_l c_l Re(rho_l conj(d rho^M_l / dgamma))
 * with d rho^M/dgamma summed image by image using d(g_top^a g_bot^b).
 */
double orc_kspace_dgamma(int64_t N, const double *pos, const double *q, const orc_box *b,
                         int P, const int32_t *n, const double *c, int which)
{
    double *rho = malloc(sizeof(double) * 2 * P);
    orc_rho(N, pos, q, b, P, n, 0, rho);
    double *dg_p = malloc(sizeof(double) * (b->M + 1));
    double *dg_m = malloc(sizeof(double) * (b->M + 1));
    for (int o = 1; o <= b->M; o++) {
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            int a, bb;
            orc_image_exponents(o, sgn, &a, &bb);
            double d;
            if (which == 0) d = a ? a * ipow(b->g_top, a - 1) * ipow(b->g_bot, bb) : 0.0;
            else            d = bb ? bb * ipow(b->g_bot, bb - 1) * ipow(b->g_top, a) : 0.0;
            if (sgn > 0) dg_p[o - 1] = d; else dg_m[o - 1] = d;
        }
    }
    double e = 0.0;
#pragma omp parallel for reduction(+ : e) schedule(static)
    for (int l = 0; l < P; l++) {
        double k[3];
        kvec(b, n + 3 * l, k);
        double re = 0, im = 0;
        for (int64_t j = 0; j < N; j++) {
            double x = pos[3 * j], y = pos[3 * j + 1], z = pos[3 * j + 2];
            for (int o = 1; o <= b->M; o++) {
                double tp = k[0] * x + k[1] * y + k[2] * orc_image_z(o, +1, z, b->H);
                double tm = k[0] * x + k[1] * y + k[2] * orc_image_z(o, -1, z, b->H);
                re += q[j] * (dg_p[o - 1] * cos(tp) + dg_m[o - 1] * cos(tm));
                im += q[j] * (dg_p[o - 1] * sin(tp) + dg_m[o - 1] * sin(tm));
            }
        }
        e += c[l] * (rho[2 * l] * re + rho[2 * l + 1] * im);
    }
    free(rho); free(dg_p); free(dg_m);
    return e;
}

/* ------------------------------------------------------------------ */
/* IBC term with images (Theorem 3.3, U_IBC^M) and self energy          */
/* ------------------------------------------------------------------ */

/*
 *   U_IBC^M = (2 pi / V) mu * muM,  mu = sum_i q_i z_i,
 *   muM = sum_j q_j [ z_j + sum_l (g+ z_j+^(l) + g- z_j-^(l)) ].
 * F (n_t x 3, z component only non-zero) = -grad (R5); phi = dU/dq_i.
 * dEdg (2, may be NULL): derivative with respect to gamma_top, gamma_bot.
 */
void orc_ibc(int64_t N, const double *pos, const double *q, const orc_box *b,
             int64_t n_t, const int64_t *tgt, double *E, double *F, double *phi,
             double *dEdg)
{
    double V = b->Lx * b->Ly * b->Lz;
    double *gp = malloc(sizeof(double) * (b->M + 1));
    double *gm = malloc(sizeof(double) * (b->M + 1));
    orc_image_coeffs(b->M, b->g_top, b->g_bot, gp, gm);
    double mu = 0.0, muM = 0.0, dmu_t = 0.0, dmu_b = 0.0;
    for (int64_t j = 0; j < N; j++) {
        double z = pos[3 * j + 2], w = z, wt = 0.0, wb = 0.0;
        for (int o = 1; o <= b->M; o++) {
            double zp = orc_image_z(o, +1, z, b->H), zm = orc_image_z(o, -1, z, b->H);
            w += gp[o - 1] * zp + gm[o - 1] * zm;
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                int a, bb;
                orc_image_exponents(o, sgn, &a, &bb);
                double zi = sgn > 0 ? zp : zm;
                if (a) wt += a * ipow(b->g_top, a - 1) * ipow(b->g_bot, bb) * zi;
                if (bb) wb += bb * ipow(b->g_bot, bb - 1) * ipow(b->g_top, a) * zi;
            }
        }
        mu += q[j] * z;
        muM += q[j] * w;
        dmu_t += q[j] * wt;
        dmu_b += q[j] * wb;
    }
    if (E) *E = 2.0 * ORC_PI / V * mu * muM;
    if (dEdg) {
        dEdg[0] = 2.0 * ORC_PI / V * mu * dmu_t;
        dEdg[1] = 2.0 * ORC_PI / V * mu * dmu_b;
    }
    /* dw_j/dz_j = 1 + sum_l (-1)^l (g+ + g-) */
    double dw = 1.0;
    for (int o = 1; o <= b->M; o++) dw += ((o % 2 == 0) ? 1.0 : -1.0) * (gp[o - 1] + gm[o - 1]);
    int64_t nt = tgt ? n_t : N;
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = tgt ? tgt[t] : t;
        double z = pos[3 * i + 2];
        if (F) {
            F[3 * t] = 0.0;
            F[3 * t + 1] = 0.0;
            F[3 * t + 2] = -2.0 * ORC_PI / V * (q[i] * muM + mu * q[i] * dw);
        }
        if (phi) {
            double w = z;
            for (int o = 1; o <= b->M; o++)
                w += gp[o - 1] * orc_image_z(o, +1, z, b->H) + gm[o - 1] * orc_image_z(o, -1, z, b->H);
            phi[t] = 2.0 * ORC_PI / V * (z * muM + mu * w);
        }
    }
    free(gp);
    free(gm);
}

/* ------------------------------------------------------------------ */
/* Surface charges on the interfaces (remark after Eq. (3.26); the     */
/* supplement it refers to is not available -- readings R7, R8 below) */
/* ------------------------------------------------------------------ */

/*
 * R7  A uniform surface charge density sigma_bot on the interface z = 0 and
 *     sigma_top on z = H are sheets of charge taken just inside the slab.
 *     Their images follow the image series of Sec. 3.1 (a sheet is a
 *     charge distribution like any other: its order-l images are sheets at
 *     the image heights with the image weights).  A uniform sheet s at
 *     height z_s has the potential -2 pi s |z - z_s| in the doubly periodic
 *     geometry (the zero lateral mode), so an ion q_i at z_i gains
 *       E = q_i phi_s(z_i),  phi_s(z) = -2 pi sum_{sheets, images} w sigma |z - z_w|,
 *       F_z = 2 pi q_i sum w sigma sign(z_i - z_w).
 * R8  With surface charges the ions are not neutral (Q = sum q_i != 0).
 *     Theorem 3.3 assumes neutrality: its k-sum over the Lz-periodic box
 *     drops k = 0.  Writing out the k_x = k_y = 0 part of that sum for the
 *     pair potential (4 pi / V) sum_{kz != 0} e^{i kz d}/kz^2 = -(2 pi/(Lx Ly))|d|
 *     + (2 pi / V) d^2 + const shows that, besides the IBC term
 *     (2 pi / V) mu mu^M, the slab energy needs
 *       U_Q = -(pi / V) sum_{i, j, images w} q_i q_j w (z_i^2 + (z_j^w)^2),
 *     which vanishes for neutral ions.  Position-independent terms are
 *     dropped, so with Q != 0 the energy is defined up to a constant (and
 *     dE/dq up to a term proportional to Q); forces are unique.
 *
 * orc_surface returns the two additions (sheet field and U_Q): the energy
 * E, the forces F (n_t x 3, z only), phi = dE/dq_i for the targets and,
 * with dEdg, dE/dgamma_{top,bot}.
 */
void orc_surface(int64_t N, const double *pos, const double *q, const orc_box *b, double sig_top,
                 double sig_bot, int64_t n_t, const int64_t *tgt, double *E, double *F, double *phi,
                 double *dEdg)
{
    double V = b->Lx * b->Ly * b->Lz;
    double *gp = malloc(sizeof(double) * (b->M + 1));
    double *gm = malloc(sizeof(double) * (b->M + 1));
    orc_image_coeffs(b->M, b->g_top, b->g_bot, gp, gm);
    /* weights and their gamma derivatives of the sources: w[0] = real, then
     * the + and - image of each order; the image heights of a charge at z
     * are z_w = s_w z + c_w with s_w = (-1)^l */
    int nw = 1 + 2 * b->M;
    double *w = malloc(sizeof(double) * nw), *dwt = malloc(sizeof(double) * nw), *dwb = malloc(sizeof(double) * nw);
    w[0] = 1.0; dwt[0] = 0.0; dwb[0] = 0.0;
    for (int o = 1; o <= b->M; o++) {
        for (int k = 0; k < 2; k++) {
            int sgn = k == 0 ? +1 : -1, a, bb;
            orc_image_exponents(o, sgn, &a, &bb);
            int idx = 2 * o - 1 + k;
            w[idx] = sgn > 0 ? gp[o - 1] : gm[o - 1];
            dwt[idx] = a ? a * ipow(b->g_top, a - 1) * ipow(b->g_bot, bb) : 0.0;
            dwb[idx] = bb ? bb * ipow(b->g_bot, bb - 1) * ipow(b->g_top, a) : 0.0;
        }
    }
#define ZW(idx, z) ((idx) == 0 ? (z) : orc_image_z(((idx) + 1) / 2, ((idx) % 2) ? +1 : -1, (z), b->H))
#define SW(idx) ((idx) == 0 ? 1.0 : ((((idx) + 1) / 2) % 2 ? -1.0 : 1.0))
    /* sums over the sources: Q^M = sum_{j,w} q_j w, QZ2 = sum_{j,w} q_j w z_j^w^2,
     * S2 = sum q z^2, Q = sum q, and their gamma derivatives */
    double Q = 0, S2 = 0, QM = 0, QZ2 = 0, dQM[2] = {0, 0}, dQZ2[2] = {0, 0};
    for (int64_t j = 0; j < N; j++) {
        double z = pos[3 * j + 2];
        Q += q[j];
        S2 += q[j] * z * z;
        for (int k = 0; k < nw; k++) {
            double zw = ZW(k, z);
            QM += q[j] * w[k];
            QZ2 += q[j] * w[k] * zw * zw;
            dQM[0] += q[j] * dwt[k]; dQM[1] += q[j] * dwb[k];
            dQZ2[0] += q[j] * dwt[k] * zw * zw; dQZ2[1] += q[j] * dwb[k] * zw * zw;
        }
    }
    double UQ = -ORC_PI / V * (S2 * QM + Q * QZ2);
    /* the two sheets (bottom at z = 0, top at z = H, from inside) and their images */
    const double zs[2] = {0.0, b->H}, sg[2] = {sig_bot, sig_top};
    double Es = 0.0, dEs[2] = {0, 0};
    for (int64_t i = 0; i < N; i++) {
        double z = pos[3 * i + 2], ph = 0.0, dph[2] = {0, 0};
        for (int s = 0; s < 2; s++)
            for (int k = 0; k < nw; k++) {
                double d = fabs(z - ZW(k, zs[s]));
                ph += -2.0 * ORC_PI * sg[s] * w[k] * d;
                dph[0] += -2.0 * ORC_PI * sg[s] * dwt[k] * d;
                dph[1] += -2.0 * ORC_PI * sg[s] * dwb[k] * d;
            }
        Es += q[i] * ph;
        dEs[0] += q[i] * dph[0];
        dEs[1] += q[i] * dph[1];
    }
    if (E) *E = UQ + Es;
    if (dEdg)
        for (int c = 0; c < 2; c++) dEdg[c] = -ORC_PI / V * (S2 * dQM[c] + Q * dQZ2[c]) + dEs[c];
    int64_t nt = tgt ? n_t : N;
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = tgt ? tgt[t] : t;
        double z = pos[3 * i + 2];
        /* d/dz_i of sum_w w z_i^w^2 = sum_w w 2 s_w z_i^w; of the sheet potential */
        double dZ2 = 0.0, Z2i = 0.0, Wi = 0.0, fs = 0.0, phs = 0.0;
        for (int k = 0; k < nw; k++) {
            double zw = ZW(k, z);
            dZ2 += w[k] * 2.0 * SW(k) * zw;
            Z2i += w[k] * zw * zw;
            Wi += w[k];
        }
        for (int s = 0; s < 2; s++)
            for (int k = 0; k < nw; k++) {
                double dz = z - ZW(k, zs[s]);
                fs += 2.0 * ORC_PI * sg[s] * w[k] * (dz > 0 ? 1.0 : (dz < 0 ? -1.0 : 0.0));
                phs += -2.0 * ORC_PI * sg[s] * w[k] * fabs(dz);
            }
        if (F) {
            F[3 * t] = 0.0;
            F[3 * t + 1] = 0.0;
            /* -d U_Q / d z_i: U_Q has q_i z_i^2 Q^M and Q q_i sum_w w z_i^w^2 */
            F[3 * t + 2] = ORC_PI / V * (2.0 * q[i] * z * QM + Q * q[i] * dZ2) + q[i] * fs;
        }
        if (phi) phi[t] = -ORC_PI / V * (z * z * QM + S2 * Wi + QZ2 + Q * Z2i) + phs;
    }
#undef ZW
#undef SW
    free(w); free(dwt); free(dwb);
    free(gp);
    free(gm);
}

/* Self-energy correction -alpha/sqrt(pi) sum q_i^2 (Eq. (3.16)). */
double orc_self(int64_t N, const double *q, double alpha)
{
    double s = 0.0;
    for (int64_t i = 0; i < N; i++) s += q[i] * q[i];
    return -alpha / sqrt(ORC_PI) * s;
}

/* ------------------------------------------------------------------ */
/* Real space with images (Eq. (3.12)), brute force over all sources    */
/* ------------------------------------------------------------------ */

static double min_image(double d, double L) { return d - L * nearbyint(d / L); }

/*
 * For each target i: phi_i = sum_s q_s w_s erfc(alpha d)/d over the sources
 * s = every other real charge (minimum image in x, y) and every image of
 * order 1..M of every charge including i itself, counted if d < rc (R6).
 * F_i = q_i sum_s q_s w_s [erfc(a d)/d + 2a/sqrt(pi) e^{-a^2 d^2}] dvec/d^2 (R5).
 * E_real = 1/2 sum_i q_i phi_i (over all particles; only when tgt == NULL).
 * dphig (n_t x 2, may be NULL): per-target d phi_i / d gamma_{top,bot}.
 */
void orc_real(int64_t N, const double *pos, const double *q, const orc_box *b,
              int64_t n_t, const int64_t *tgt, double *E, double *F, double *phi,
              double *dphig)
{
    double *gp = malloc(sizeof(double) * (b->M + 1));
    double *gm = malloc(sizeof(double) * (b->M + 1));
    orc_image_coeffs(b->M, b->g_top, b->g_bot, gp, gm);
    const double a = b->alpha, rc = b->rc;
    const double c2 = 2.0 * a / sqrt(ORC_PI);
    int64_t nt = tgt ? n_t : N;
    double *ph = malloc(sizeof(double) * (nt > 0 ? nt : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = tgt ? tgt[t] : t;
        double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        double fx = 0, fy = 0, fz = 0, p = 0, pt = 0, pb = 0;
        for (int64_t j = 0; j < N; j++) {
            double dx = min_image(xi - pos[3 * j], b->Lx);
            double dy = min_image(yi - pos[3 * j + 1], b->Ly);
            double zj = pos[3 * j + 2];
            for (int o = 0; o <= b->M; o++) {
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    double w, zs;
                    int ea = 0, eb = 0;
                    if (o == 0) {
                        if (sgn > 0) continue;          /* the real charge, once */
                        if (j == i) continue;           /* excluded self term */
                        w = 1.0;
                        zs = zj;
                    } else {
                        w = sgn > 0 ? gp[o - 1] : gm[o - 1];
                        zs = orc_image_z(o, sgn, zj, b->H);
                        orc_image_exponents(o, sgn, &ea, &eb);
                    }
                    double dz = zi - zs;
                    if (fabs(dz) >= rc) continue;
                    double d2 = dx * dx + dy * dy + dz * dz;
                    double d = sqrt(d2);
                    if (!(d < rc)) continue;
                    double ec = erfc(a * d) / d;
                    double s = q[j] * w * (ec + c2 * exp(-a * a * d2)) / d2;
                    fx += s * dx;
                    fy += s * dy;
                    fz += s * dz;
                    p += q[j] * w * ec;
                    if (o > 0) {
                        if (ea) pt += q[j] * ea * ipow(b->g_top, ea - 1) * ipow(b->g_bot, eb) * ec;
                        if (eb) pb += q[j] * eb * ipow(b->g_bot, eb - 1) * ipow(b->g_top, ea) * ec;
                    }
                }
            }
        }
        if (F) {
            F[3 * t] = q[i] * fx;
            F[3 * t + 1] = q[i] * fy;
            F[3 * t + 2] = q[i] * fz;
        }
        ph[t] = p;
        if (phi) phi[t] = p;
        if (dphig) { dphig[2 * t] = pt; dphig[2 * t + 1] = pb; }
    }
    if (E) {
        double e = 0.0;
        if (!tgt)
            for (int64_t i = 0; i < N; i++) e += 0.5 * q[i] * ph[i];
        *E = e;
    }
    free(ph);
    free(gp);
    free(gm);
}

/* ------------------------------------------------------------------ */
/* Short-range forces of the MD around the path (Sec. 4.1): purely      */
/* repulsive shifted-truncated LJ between ions (cut at 2^(1/6) sigma,   */
/* shifted by +eps so that it vanishes there), and the same form in the */
/* distance to each wall (z = 0 and z = H) with sigma_w, eps_w (reading: */
/* the wall form is not printed).  Brute force over all pairs, minimum  */
/* image in x and y.                                                    */
/* ------------------------------------------------------------------ */

static double lj_shifted(double s2_over_r2, double eps, double *f_over_r2_times_r2)
{
    /* returns U; *f... = -dU/dr * r (i.e. r * |F|) */
    double s6 = s2_over_r2 * s2_over_r2 * s2_over_r2;
    *f_over_r2_times_r2 = 24.0 * eps * (2.0 * s6 * s6 - s6);
    return 4.0 * eps * (s6 * s6 - s6 + 0.25);
}

void orc_short(int64_t N, const double *pos, double Lx, double Ly, double H, double sigma, double eps,
               double sigma_w, double eps_w, double *F, double *E_pair, double *E_wall)
{
    const double rcut2 = pow(2.0, 1.0 / 3.0) * sigma * sigma;
    const double hcut = pow(2.0, 1.0 / 6.0) * sigma_w;
    double ep = 0.0, ew = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : ep, ew)
    for (int64_t i = 0; i < N; i++) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
        if (eps != 0.0) {
            for (int64_t j = 0; j < N; j++) {
                if (j == i) continue;
                double dx = pos[3 * i] - pos[3 * j];
                double dy = pos[3 * i + 1] - pos[3 * j + 1];
                double dz = pos[3 * i + 2] - pos[3 * j + 2];
                dx -= Lx * rint(dx / Lx);
                dy -= Ly * rint(dy / Ly);
                double r2 = dx * dx + dy * dy + dz * dz;
                if (!(r2 < rcut2)) continue;
                double rf;
                double u = lj_shifted(sigma * sigma / r2, eps, &rf);
                fx += rf / r2 * dx;
                fy += rf / r2 * dy;
                fz += rf / r2 * dz;
                ep += 0.5 * u;
            }
        }
        if (eps_w != 0.0) {
            double z = pos[3 * i + 2];
            double h[2] = {z, H - z};
            double sgn[2] = {1.0, -1.0};
            for (int w = 0; w < 2; w++) {
                if (!(h[w] > 0.0 && h[w] < hcut)) continue;
                double rf;
                double u = lj_shifted(sigma_w * sigma_w / (h[w] * h[w]), eps_w, &rf);
                fz += sgn[w] * rf / h[w];
                ew += u;
            }
        }
        F[3 * i] = fx;
        F[3 * i + 1] = fy;
        F[3 * i + 2] = fz;
    }
    if (E_pair) *E_pair = ep;
    if (E_wall) *E_wall = ew;
}

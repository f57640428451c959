/*
 * lbm_oracle.c -- plain FP64 CPU oracle for the lattice Boltzmann stream-collide
 * path.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this file; the product library never does.
 *
 * What it computes follows the paper's statement of the method (Section 2,
 * "The Lattice Boltzmann Method", Eq. (1) collision and Eq. (2) streaming),
 * with the collision operator read as a two-relaxation-time (TRT) operator
 * (the paper's D3Q19 "Double Relaxation Time" scheme of the LaBS section) or
 * as a multiple-relaxation-time operator in a moment space (the LAGOON
 * collision, Section 5.2), Guo body forcing, halfway bounce-back walls,
 * velocity and pressure faces, solid cells and periodic faces.  The memory
 * layout is deliberately different from the GPU path: two full lattices and a
 * push (scatter) streaming step, one loop nest per time step, no fusion
 * beyond what Eq. (1)-(2) state.
 *
 * Everything is FP64.  The optional BF16 switch of the MLP routines emulates
 * the rounding of operands to bfloat16 (round to nearest even) so that the
 * GPU inference can be compared at its own precision; accumulation stays FP64.
 *
 * Parity status of each function is stated in its comment ("pinned by ...").
 * Functions without such a pin say "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Velocity sets.  Pairs are (odd, odd+1): direction i and its opposite.     */
/* D3Q19: rest, 6 face neighbours, 12 edge neighbours.                       */
/* D3Q27: D3Q19 plus the 8 corner neighbours.                                */
/* Weights: D3Q19 1/3, 1/18, 1/36.  D3Q27 8/27, 2/27, 1/54, 1/216.           */
/* Pinned by the exact moment identities of the velocity set (tests).        */
/* ------------------------------------------------------------------------ */
static const int VEL[27][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},
    {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1},  {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1},
};

static double weight(int q, int i)
{
    int n = abs(VEL[i][0]) + abs(VEL[i][1]) + abs(VEL[i][2]);
    if (q == 19) {
        if (n == 0) return 1.0 / 3.0;
        if (n == 1) return 1.0 / 18.0;
        return 1.0 / 36.0;
    }
    if (n == 0) return 8.0 / 27.0;
    if (n == 1) return 2.0 / 27.0;
    if (n == 2) return 1.0 / 54.0;
    return 1.0 / 216.0;
}

static int opposite(int i)
{
    if (i == 0) return 0;
    return (i % 2 == 1) ? i + 1 : i - 1;
}

/* Copy the velocity set out for the tests: c[q][3], w[q], opp[q]. */
int orc_velocity_set(int q, int *c, double *w, int *opp)
{
    if (q != 19 && q != 27) return -1;
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = VEL[i][a];
        w[i] = weight(q, i);
        opp[i] = opposite(i);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium: second-order polynomial in u on both lattices,              */
/*   f_i^eq = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u),  c_s^2 = 1/3.     */
/* Pinned by its moments rho, rho u, rho/3 I + rho u u (tests).              */
/* ------------------------------------------------------------------------ */
void orc_equilibrium(int q, double rho, const double *u, double *feq)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < q; ++i) {
        double cu = VEL[i][0] * u[0] + VEL[i][1] * u[1] + VEL[i][2] * u[2];
        feq[i] = weight(q, i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* ------------------------------------------------------------------------ */
/* Guo forcing term S_i = w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)].           */
/* Pinned through the collision invariants (momentum gains exactly F).      */
/* ------------------------------------------------------------------------ */
static void guo_source(int q, const double *u, const double *F, double *S)
{
    for (int i = 0; i < q; ++i) {
        double cu = VEL[i][0] * u[0] + VEL[i][1] * u[1] + VEL[i][2] * u[2];
        double cF = VEL[i][0] * F[0] + VEL[i][1] * F[1] + VEL[i][2] * F[2];
        double cmuF = (VEL[i][0] - u[0]) * F[0] + (VEL[i][1] - u[1]) * F[1] + (VEL[i][2] - u[2]) * F[2];
        S[i] = weight(q, i) * (3.0 * cmuF + 9.0 * cu * cF);
    }
}

/* ------------------------------------------------------------------------ */
/* Multiple-relaxation-time (MRT) collision: relaxation in a moment space.   */
/* The moments are polynomials of the lattice velocity; each moment relaxes   */
/* toward the moment of f^eq with its own rate.                               */
/*   D3Q19: the 19 polynomial moments 1, 19|c|^2-30, (21|c|^4-53|c|^2+24)/2,  */
/*   c_a, (5|c|^2-9) c_a, 3c_x^2-|c|^2, (3|c|^2-5)(3c_x^2-|c|^2), c_y^2-c_z^2, */
/*   (3|c|^2-5)(c_y^2-c_z^2), c_x c_y, c_y c_z, c_x c_z,                      */
/*   (c_y^2-c_z^2) c_x, (c_z^2-c_x^2) c_y, (c_x^2-c_y^2) c_z.                 */
/*   D3Q27: the 27 products T_a(c_x) T_b(c_y) T_c(c_z), T_0 = 1, T_1 = c,     */
/*   T_2 = 3c^2 - 2.                                                          */
/* Rate groups: 0 conserved density, 1 momentum (no effect with the Guo       */
/* source), 2 viscous (second-order deviatoric moments, rate 1/tau),          */
/* and the "ghost" groups 3 energy, 4 energy square, 5 heat flux q,           */
/* 6 pi (fourth order), 7 m (third-order anti-symmetric).  Pinned by the      */
/* orthogonality of the bases, the BGK and TRT special cases, conservation    */
/* and the Poiseuille and Taylor-Green flows (tests).                         */
/* ------------------------------------------------------------------------ */
enum { G_RHO = 0, G_J = 1, G_NU = 2, G_E = 3, G_EPS = 4, G_Q = 5, G_PI = 6, G_M = 7 };

static double mrt_moment19(int a, const int *c, int *group)
{
    double x = c[0], y = c[1], z = c[2], c2 = x * x + y * y + z * z;
    switch (a) {
    case 0: *group = G_RHO; return 1.0;
    case 1: *group = G_E; return 19.0 * c2 - 30.0;
    case 2: *group = G_EPS; return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: *group = G_J; return x;
    case 4: *group = G_Q; return (5.0 * c2 - 9.0) * x;
    case 5: *group = G_J; return y;
    case 6: *group = G_Q; return (5.0 * c2 - 9.0) * y;
    case 7: *group = G_J; return z;
    case 8: *group = G_Q; return (5.0 * c2 - 9.0) * z;
    case 9: *group = G_NU; return 3.0 * x * x - c2;
    case 10: *group = G_PI; return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
    case 11: *group = G_NU; return y * y - z * z;
    case 12: *group = G_PI; return (3.0 * c2 - 5.0) * (y * y - z * z);
    case 13: *group = G_NU; return x * y;
    case 14: *group = G_NU; return y * z;
    case 15: *group = G_NU; return x * z;
    case 16: *group = G_M; return (y * y - z * z) * x;
    case 17: *group = G_M; return (z * z - x * x) * y;
    default: *group = G_M; return (x * x - y * y) * z;
    }
}

static double cheb(int k, double c) { return k == 0 ? 1.0 : (k == 1 ? c : 3.0 * c * c - 2.0); }

static double mrt_moment27(int a, const int *c, int *group)
{
    int kx = a % 3, ky = (a / 3) % 3, kz = a / 9;
    int ones = (kx == 1) + (ky == 1) + (kz == 1), twos = (kx == 2) + (ky == 2) + (kz == 2);
    int order = ones + 2 * twos;
    if (order == 0) *group = G_RHO;
    else if (order == 1) *group = G_J;
    else if (order == 2) *group = G_NU;        /* c_a c_b and T_2(c_a) */
    else if (order == 3) *group = G_Q;         /* c_a T_2(c_b), c_x c_y c_z */
    else if (order == 4) *group = (ones == 0) ? G_E : G_PI;  /* T_2 T_2 ; c_a c_b T_2(c_c) */
    else if (order == 5) *group = G_M;
    else *group = G_EPS;                       /* T_2 T_2 T_2 */
    return cheb(kx, c[0]) * cheb(ky, c[1]) * cheb(kz, c[2]);
}

/* Moment matrix M[a][i] and the rate group of each row; returns 0 on success. */
int orc_mrt_basis(int q, double *M, int *groups)
{
    if (q != 19 && q != 27) return -1;
    for (int a = 0; a < q; ++a)
        for (int i = 0; i < q; ++i) {
            int g;
            M[a * q + i] = q == 19 ? mrt_moment19(a, VEL[i], &g) : mrt_moment27(a, VEL[i], &g);
            groups[a] = g;
        }
    return 0;
}

/* Inverse of an n x n matrix by Gauss-Jordan elimination with partial     */
/* pivoting; returns 0 on success, -1 if singular.                         */
static int invert(int n, const double *A, double *Ainv)
{
    double W[27 * 54];
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < 2 * n; ++k) W[r * 2 * n + k] = k < n ? A[r * n + k] : (k - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(W[r * 2 * n + col]) > fabs(W[piv * 2 * n + col])) piv = r;
        if (fabs(W[piv * 2 * n + col]) < 1e-12) return -1;
        if (piv != col)
            for (int k = 0; k < 2 * n; ++k) {
                double t = W[col * 2 * n + k];
                W[col * 2 * n + k] = W[piv * 2 * n + k];
                W[piv * 2 * n + k] = t;
            }
        double d = W[col * 2 * n + col];
        for (int k = 0; k < 2 * n; ++k) W[col * 2 * n + k] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = W[r * 2 * n + col];
            if (f == 0.0) continue;
            for (int k = 0; k < 2 * n; ++k) W[r * 2 * n + k] -= f * W[col * 2 * n + k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int k = 0; k < n; ++k) Ainv[r * n + k] = W[r * 2 * n + n + k];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Closure parameters and the MLP (6 -> 32 -> 32 -> 1).                     */
/* ------------------------------------------------------------------------ */
enum { CL_NONE = 0, CL_SMAG = 1, CL_MLP = 2 };
enum { MLP_IN = 6, MLP_H = 32 };
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1) /* 1313 */
#define MLP_NNORM (4 * MLP_IN)                                                 /* mu, sigma, lo, hi */

/* Round a double to the nearest bfloat16 value (ties to even), via float.   */
/* Pinned against torch's float -> bfloat16 conversion (tests).              */
double orc_round_bf16(double x)
{
    float f = (float)x;
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan */
    uint32_t lsb = (b >> 16) & 1u;
    b += 0x7fffu + lsb;
    b &= 0xffff0000u;
    memcpy(&f, &b, 4);
    return (double)f;
}

static double rnd(double x, int bf16) { return bf16 ? orc_round_bf16(x) : x; }

static double softplus(double o) { return o > 30.0 ? o : log1p(exp(o)); }

/*
 * MLP forward for one input vector x[6] (already raw features).  Layout of
 * params: W1[32][6], b1[32], W2[32][32], b2[32], W3[32], b3.  Inputs are
 * standardised with norm = {mu[6], sigma[6], lo[6], hi[6]}.  Hidden layers
 * use tanh; the output passes through softplus so the correction is >= 0.
 * With bf16 != 0, every matrix operand (inputs and weights of each layer)
 * is rounded to bfloat16 first; sums, biases and activations are FP64.
 * Returns the relaxation-time correction; h1, h2 (nullable) receive the
 * hidden activations, o_out the pre-softplus output.
 * Pinned by finite differences of its backward pass and by closed-form
 * single-unit cases (tests).
 */
double orc_mlp_forward1(const double *params, const double *norm, const double *x, int bf16,
                        double *h1_out, double *h2_out, double *o_out)
{
    const double *W1 = params;
    const double *b1 = W1 + MLP_H * MLP_IN;
    const double *W2 = b1 + MLP_H;
    const double *b2 = W2 + MLP_H * MLP_H;
    const double *W3 = b2 + MLP_H;
    const double *b3 = W3 + MLP_H;
    double z[MLP_IN], h1[MLP_H], h2[MLP_H];
    for (int k = 0; k < MLP_IN; ++k) z[k] = (x[k] - norm[k]) / norm[MLP_IN + k];
    for (int j = 0; j < MLP_H; ++j) {
        double s = 0.0;
        for (int k = 0; k < MLP_IN; ++k) s += rnd(W1[j * MLP_IN + k], bf16) * rnd(z[k], bf16);
        h1[j] = tanh(s + b1[j]);
    }
    for (int j = 0; j < MLP_H; ++j) {
        double s = 0.0;
        for (int k = 0; k < MLP_H; ++k) s += rnd(W2[j * MLP_H + k], bf16) * rnd(h1[k], bf16);
        h2[j] = tanh(s + b2[j]);
    }
    double o = b3[0];
    {
        double s = 0.0;
        for (int k = 0; k < MLP_H; ++k) s += rnd(W3[k], bf16) * rnd(h2[k], bf16);
        o += s;
    }
    if (h1_out) memcpy(h1_out, h1, sizeof h1);
    if (h2_out) memcpy(h2_out, h2, sizeof h2);
    if (o_out) *o_out = o;
    return softplus(o);
}

/* Batched forward: x[n][6] -> y[n].  Pinned as orc_mlp_forward1. */
void orc_mlp_forward(const double *params, const double *norm, const double *x, int64_t n, int bf16,
                     double *y)
{
    for (int64_t r = 0; r < n; ++r) y[r] = orc_mlp_forward1(params, norm, x + 6 * r, bf16, 0, 0, 0);
}

/*
 * Loss and gradient for a batch: loss = (1/n) sum_r (y_r - t_r)^2 with y the
 * MLP output.  grad[1313] receives d loss / d params (plain FP64 backward by
 * the chain rule through softplus, the two tanh layers and the affine maps).
 * Returns the loss.  Pinned by central finite differences (tests).
 */
double orc_mlp_loss_grad(const double *params, const double *norm, const double *x, const double *t,
                         int64_t n, double *grad)
{
    const double *W2 = params + MLP_H * MLP_IN + MLP_H;
    const double *W3 = W2 + MLP_H * MLP_H + MLP_H;
    double *gW1 = grad;
    double *gb1 = gW1 + MLP_H * MLP_IN;
    double *gW2 = gb1 + MLP_H;
    double *gb2 = gW2 + MLP_H * MLP_H;
    double *gW3 = gb2 + MLP_H;
    double *gb3 = gW3 + MLP_H;
    memset(grad, 0, sizeof(double) * MLP_NPARAM);
    double loss = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        const double *xr = x + 6 * r;
        double h1[MLP_H], h2[MLP_H], o, z[MLP_IN];
        double y = orc_mlp_forward1(params, norm, xr, 0, h1, h2, &o);
        for (int k = 0; k < MLP_IN; ++k) z[k] = (xr[k] - norm[k]) / norm[MLP_IN + k];
        double e = y - t[r];
        loss += e * e;
        /* d loss_r / d y = 2 e / n ; softplus'(o) = logistic(o) */
        double dy = 2.0 * e / (double)n;
        double dout = dy / (1.0 + exp(-o));
        gb3[0] += dout;
        double d2[MLP_H];
        for (int k = 0; k < MLP_H; ++k) {
            gW3[k] += dout * h2[k];
            d2[k] = dout * W3[k] * (1.0 - h2[k] * h2[k]);
        }
        double d1[MLP_H];
        for (int k = 0; k < MLP_H; ++k) d1[k] = 0.0;
        for (int j = 0; j < MLP_H; ++j) {
            gb2[j] += d2[j];
            for (int k = 0; k < MLP_H; ++k) {
                gW2[j * MLP_H + k] += d2[j] * h1[k];
                d1[k] += d2[j] * W2[j * MLP_H + k];
            }
        }
        for (int k = 0; k < MLP_H; ++k) d1[k] *= (1.0 - h1[k] * h1[k]);
        for (int j = 0; j < MLP_H; ++j) {
            gb1[j] += d1[j];
            for (int k = 0; k < MLP_IN; ++k) gW1[j * MLP_IN + k] += d1[j] * z[k];
        }
    }
    return loss / (double)n;
}

/*
 * One Adam update (Kingma & Ba, 2015) of p[n] with gradient g[n] and moment
 * buffers m[n], v[n]; step is the 1-based update count.
 * Pinned by the closed form of the first update (|dp| = lr for every
 * non-zero gradient component) in the tests.
 */
void orc_adam(double *p, const double *g, double *m, double *v, int64_t n, int64_t step, double lr,
              double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)step);
    double c2 = 1.0 - pow(beta2, (double)step);
    for (int64_t k = 0; k < n; ++k) {
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
        double mh = m[k] / c1, vh = v[k] / c2;
        p[k] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Smagorinsky closure in the Hou et al. (1996) form.                        */
/* tau_tot solves tau_tot^2 - tau tau_tot - (9 sqrt2 / 2) Cs^2 Q / rho = 0,  */
/* Q = |P_c| (Frobenius norm of the non-equilibrium momentum flux).          */
/* Pinned by the residual of that quadratic and by Cs = 0 -> tau (tests).    */
/* ------------------------------------------------------------------------ */
double orc_smagorinsky_tau(double tau, double cs, double Q, double rho)
{
    return 0.5 * (tau + sqrt(tau * tau + 18.0 * sqrt(2.0) * cs * cs * Q / rho));
}

/*
 * The six local features of a cell given its non-equilibrium flux per unit
 * density P (symmetric 3x3, packed xx, yy, zz, xy, xz, yz), its density and
 * the molecular tau:
 *   x1 = tr P,  x2 = |P_dev|_F,  x3 = cbrt(det P_dev),  x4 = rho - 1,
 *   x5 = tau_smag - tau (Cs of the domain, Q = rho |P|),  x6 = tau.
 * Pinned by invariance under rotations and closed forms for diagonal P
 * (tests).
 */
void orc_features(const double *P, double rho, double tau, double cs, double *xo)
{
    double tr = P[0] + P[1] + P[2];
    double d0 = P[0] - tr / 3.0, d1 = P[1] - tr / 3.0, d2 = P[2] - tr / 3.0;
    double xy = P[3], xz = P[4], yz = P[5];
    double nd = sqrt(d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * (xy * xy + xz * xz + yz * yz));
    double det = d0 * (d1 * d2 - yz * yz) - xy * (xy * d2 - yz * xz) + xz * (xy * yz - d1 * xz);
    double np = sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2] + 2.0 * (xy * xy + xz * xz + yz * yz));
    xo[0] = tr;
    xo[1] = nd;
    xo[2] = cbrt(det);
    xo[3] = rho - 1.0;
    xo[4] = orc_smagorinsky_tau(tau, cs, rho * np, rho) - tau;
    xo[5] = tau;
}

/* ------------------------------------------------------------------------ */
/* Hybrid recursive regularisation (HRR; Jacob, Malaspinas & Sagaut 2018:    */
/* the "D3Q19HRR" collision of the LaBS section).  D3Q19 only.               */
/* The post-collision state is rebuilt from Hermite coefficients:            */
/*   f*_i = feq_i + (1 - 1/tau) f1_i + S_i / 2,                              */
/*   f1_i = w_i [ H2_i : Pi / (2 c_s^4) + sum_k T_k(c_i) A_k / N_k ],        */
/* the regularised form of g = f - feq + S/2 (BGK with Guo forcing written   */
/* as feq + (1 - 1/tau) g + S/2; g has no first moment, so the collision     */
/* keeps mass and adds exactly F to the momentum).  Pi = sigma Pi_PR +       */
/* (1 - sigma) Pi_FD blends the projected flux of g,                         */
/* Pi_PR = sum c c (f - feq) + (uF + Fu)/2, with the                         */
/* finite-difference one Pi_FD = -2 rho c_s^2 tau S (S the strain rate of    */
/* the velocity field), and the third-order coefficients follow by the       */
/* recursion a3_abg = u_a Pi_bg + u_b Pi_ag + u_g Pi_ab.  D3Q19 carries the   */
/* mixed third-order Hermite polynomials H_aab only as the six sums and      */
/* differences T_k (H_xxy +- H_yzz, H_xzz +- H_xyy, H_yyz +- H_xxz), which   */
/* are orthogonal with the lattice weights; A_k is the matching combination  */
/* of a3, and N_k = sum_i w_i T_k(c_i)^2 its lattice norm (the projection     */
/* reproduces the moment A_k exactly).  The equilibrium adds the same        */
/* third-order terms with a3 = rho u u u.                                    */
/* Pinned by conservation, the BGK limit (sigma = 1, u = 0, second-order     */
/* non-equilibrium), the removal of the fourth-order moments, the Taylor-    */
/* Green rate and the convergence of the Poiseuille profile (tests).         */
/* ------------------------------------------------------------------------ */
static double hermite3(const int *c, int a, int b, int g)
{
    const double cs2 = 1.0 / 3.0;
    return c[a] * c[b] * c[g] - cs2 * (c[a] * (b == g) + c[b] * (a == g) + c[g] * (a == b));
}

/* T_k(c) for k = 0..5 */
static void t3_values(const int *c, double *T)
{
    enum { X = 0, Y = 1, Z = 2 };
    double xxy = hermite3(c, X, X, Y), yzz = hermite3(c, Y, Z, Z);
    double xzz = hermite3(c, X, Z, Z), xyy = hermite3(c, X, Y, Y);
    double yyz = hermite3(c, Y, Y, Z), xxz = hermite3(c, X, X, Z);
    T[0] = xxy + yzz;
    T[1] = xxy - yzz;
    T[2] = xzz + xyy;
    T[3] = xzz - xyy;
    T[4] = yyz + xxz;
    T[5] = yyz - xxz;
}

/* The combinations A_k of a symmetric third-order tensor given by its six  */
/* mixed components a_xxy, a_yzz, a_xzz, a_xyy, a_yyz, a_xxz.               */
static void t3_combos(double xxy, double yzz, double xzz, double xyy, double yyz, double xxz, double *A)
{
    A[0] = xxy + yzz;
    A[1] = xxy - yzz;
    A[2] = xzz + xyy;
    A[3] = xzz - xyy;
    A[4] = yyz + xxz;
    A[5] = yyz - xxz;
}

/* Third-order terms of the HRR equilibrium, added to feq (a3 = rho u u u). */
static void hrr_equilibrium3(int q, double rho, const double *u, const double *norm, double *feq)
{
    double A[6], T[6];
    double x = u[0], y = u[1], z = u[2];
    t3_combos(rho * x * x * y, rho * y * z * z, rho * x * z * z, rho * x * y * y, rho * y * y * z, rho * x * x * z, A);
    for (int i = 0; i < q; ++i) {
        t3_values(VEL[i], T);
        double acc = 0.0;
        for (int k = 0; k < 6; ++k) acc += T[k] * A[k] / norm[k];
        feq[i] += weight(q, i) * acc;
    }
}

/* Regularised non-equilibrium f1 from the blended flux Pi[3][3] and u.     */
static void hrr_f1(int q, const double Pi[3][3], const double *u, const double *norm, double *f1)
{
    const double cs2 = 1.0 / 3.0;
    double a3[3][3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int g = 0; g < 3; ++g) a3[a][b][g] = u[a] * Pi[b][g] + u[b] * Pi[a][g] + u[g] * Pi[a][b];
    double A[6], T[6];
    t3_combos(a3[0][0][1], a3[1][2][2], a3[0][2][2], a3[0][1][1], a3[1][1][2], a3[0][0][2], A);
    for (int i = 0; i < q; ++i) {
        double h2 = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) h2 += (VEL[i][a] * VEL[i][b] - cs2 * (a == b)) * Pi[a][b];
        t3_values(VEL[i], T);
        double t3 = 0.0;
        for (int k = 0; k < 6; ++k) t3 += T[k] * A[k] / norm[k];
        f1[i] = weight(q, i) * (h2 / (2.0 * cs2 * cs2) + t3);
    }
}

/* Lattice norms N_k of the D3Q19 third-order combinations (2/27 for the     */
/* sums, 6/27 for the differences; pinned in the tests).                    */
int orc_hrr_norms(double *norm)
{
    double T[6];
    for (int k = 0; k < 6; ++k) norm[k] = 0.0;
    for (int i = 0; i < 19; ++i) {
        t3_values(VEL[i], T);
        for (int k = 0; k < 6; ++k) norm[k] += weight(19, i) * T[k] * T[k];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Simulation state.                                                         */
/* ------------------------------------------------------------------------ */
/* BC_INTERFACE: a face of a 2:1 refinement interface (orc_refine_step); within */
/* one lattice it returns populations as a no-slip face does.                  */
enum { BC_PERIODIC = 0, BC_NOSLIP = 1, BC_VELOCITY = 2, BC_PRESSURE = 3, BC_INTERFACE = 4 };

typedef struct {
    int q, nx, ny, nz;
    int64_t n;
    int bc[6];
    double ubc[6][3];
    double rhobc[6];
    double tau, magic, F[3];
    int closure;
    double cs;
    double mlp[MLP_NPARAM];
    double norm[MLP_NNORM];
    int collision;        /* 0 TRT, 1 MRT, 2 HRR */
    double mrt_rates[5];  /* ghost rates: energy, energy square, q, pi, m */
    double hrr_sigma;     /* HRR: weight of the projected flux (1 - weight of the FD one) */
    double t3norm[6];     /* HRR: lattice norms sum_i w_i T_k(c_i)^2 of the third-order combinations */
    double *uprev;        /* HRR: [3][n] velocity field of the previous step (the FD gradient's input) */
    double Mm[27 * 27], Minv[27 * 27];
    int mgroup[27];
    unsigned char *solid; /* NULL: all fluid */
    double *f, *g;        /* [q][n] canonical (post-stream, pre-collide) and scratch */
    int64_t fallbacks;    /* cells where the MLP closure fell back to Smagorinsky */
} orc_sim;

static void hrr_update_velocity(orc_sim *s);

static int64_t cell_index(const orc_sim *s, int x, int y, int z)
{
    return ((int64_t)z * s->ny + y) * s->nx + x;
}

static int is_solid(const orc_sim *s, int64_t c) { return s->solid ? s->solid[c] != 0 : 0; }

/*
 * Create a simulation.  bc[6] for faces -x,+x,-y,+y,-z,+z; ubc[6][3] wall
 * velocities of velocity faces; rhobc[6] wall densities of velocity and
 * pressure faces; solid (nullable) one byte per cell, non-zero = solid.
 * Returns NULL on invalid arguments.
 */
orc_sim *orc_create(int q, int nx, int ny, int nz, const int *bc, const double *ubc, const double *rhobc,
                    const unsigned char *solid, double tau, double magic, const double *F, int closure,
                    double cs)
{
    if ((q != 19 && q != 27) || nx <= 0 || ny <= 0 || nz <= 0 || tau <= 0.5) return NULL;
    for (int a = 0; a < 3; ++a)
        if ((bc[2 * a] == BC_PERIODIC) != (bc[2 * a + 1] == BC_PERIODIC)) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->q = q;
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->n = (int64_t)nx * ny * nz;
    for (int k = 0; k < 6; ++k) {
        s->bc[k] = bc[k];
        for (int a = 0; a < 3; ++a) s->ubc[k][a] = ubc ? ubc[3 * k + a] : 0.0;
        s->rhobc[k] = rhobc ? rhobc[k] : 1.0;
    }
    s->tau = tau;
    s->magic = magic;
    for (int a = 0; a < 3; ++a) s->F[a] = F ? F[a] : 0.0;
    s->closure = closure;
    s->cs = cs;
    if (solid) {
        s->solid = (unsigned char *)malloc((size_t)s->n);
        memcpy(s->solid, solid, (size_t)s->n);
    }
    /* the two lattices are allocated on first use, so that a probe-only */
    /* simulation of a large domain holds no population arrays           */
    return s;
}

static void ensure_lattices(orc_sim *s)
{
    if (!s->f) s->f = (double *)calloc((size_t)(s->q * s->n), sizeof(double));
    if (!s->g) s->g = (double *)calloc((size_t)(s->q * s->n), sizeof(double));
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->solid);
    free(s->uprev);
    free(s->f);
    free(s->g);
    free(s);
}

/* Select the MRT collision with ghost rates {s_e, s_eps, s_q, s_pi, s_m};  */
/* the viscous rate stays 1/tau (or the closure's).  Returns -1 if the      */
/* basis is singular.                                                        */
int orc_set_mrt(orc_sim *s, const double *rates)
{
    orc_mrt_basis(s->q, s->Mm, s->mgroup);
    if (invert(s->q, s->Mm, s->Minv) != 0) return -1;
    for (int k = 0; k < 5; ++k) s->mrt_rates[k] = rates[k];
    s->collision = 1;
    return 0;
}

void orc_set_mlp(orc_sim *s, const double *params, const double *norm)
{
    memcpy(s->mlp, params, sizeof(s->mlp));
    memcpy(s->norm, norm, sizeof(s->norm));
}

int64_t orc_fallbacks(const orc_sim *s) { return s->fallbacks; }

/* Set the state to f^eq(rho, u) at every fluid cell; u is [3][n].  Solid   */
/* cells hold zeros.                                                         */
void orc_init_equilibrium(orc_sim *s, const double *rho, const double *u)
{
    double feq[27], uc[3];
    ensure_lattices(s);
    for (int64_t c = 0; c < s->n; ++c) {
        for (int a = 0; a < 3; ++a) uc[a] = u[a * s->n + c];
        orc_equilibrium(s->q, rho[c], uc, feq);
        for (int i = 0; i < s->q; ++i) s->f[i * s->n + c] = is_solid(s, c) ? 0.0 : feq[i];
    }
    hrr_update_velocity(s);
}

void orc_set_pdfs(orc_sim *s, const double *f)
{
    ensure_lattices(s);
    memcpy(s->f, f, sizeof(double) * s->q * s->n);
    hrr_update_velocity(s);
}

void orc_get_pdfs(orc_sim *s, double *f)
{
    ensure_lattices(s);
    memcpy(f, s->f, sizeof(double) * s->q * s->n);
}

/*
 * Collide one cell: f[q] in, fstar[q] out; u_out receives the cell velocity
 * u = (j + F/2) / rho; tau_out the relaxation time used.  This is Eq. (1)
 * with the relaxation split over the symmetric and antisymmetric parts of
 * each pair (i, opposite(i)):
 *   f*_i = f_i - w+ (f+_i - eq+_i) - w- (f-_i - eq-_i) + (1 - w+/2) S+_i + (1 - w-/2) S-_i
 * with w+ = 1/tau and w- = 1 / (1/2 + magic / (tau - 1/2)).
 * Pinned by: mass and momentum invariants, the BGK special case, the exact
 * Poiseuille profile and the Taylor-Green decay rate (tests).
 */
static void collide_cell(const orc_sim *s, const double *f, const double (*grad)[3], double *fstar, double *u_out,
                         double *tau_out, int64_t *fallback)
{
    int q = s->q;
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < q; ++i) {
        rho += f[i];
        for (int a = 0; a < 3; ++a) j[a] += VEL[i][a] * f[i];
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * s->F[a]) / rho;
    double feq[27], S[27];
    orc_equilibrium(q, rho, u, feq);
    guo_source(q, u, s->F, S);

    double tau = s->tau;
    if (s->closure != CL_NONE) {
        /* Non-equilibrium momentum flux with the forcing correction:        */
        /* P_c = sum_i c_i c_i (f_i - feq_i) + (u F + F u) / 2                */
        double Pc[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int i = 0; i < q; ++i) acc += VEL[i][a] * VEL[i][b] * (f[i] - feq[i]);
                Pc[a][b] = acc + 0.5 * (u[a] * s->F[b] + s->F[a] * u[b]);
            }
        double Q = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Q += Pc[a][b] * Pc[a][b];
        Q = sqrt(Q);
        double tau_smag = orc_smagorinsky_tau(s->tau, s->cs, Q, rho);
        if (s->closure == CL_SMAG) {
            tau = tau_smag;
        } else {
            double P[6] = {Pc[0][0] / rho, Pc[1][1] / rho, Pc[2][2] / rho,
                           Pc[0][1] / rho, Pc[0][2] / rho, Pc[1][2] / rho};
            double x[6];
            orc_features(P, rho, s->tau, s->cs, x);
            int inside = 1;
            for (int k = 0; k < 6; ++k)
                if (!(x[k] >= s->norm[2 * MLP_IN + k] && x[k] <= s->norm[3 * MLP_IN + k])) inside = 0;
            double dt = inside ? orc_mlp_forward1(s->mlp, s->norm, x, 1, 0, 0, 0) : NAN;
            if (inside && isfinite(dt)) {
                tau = s->tau + dt;
            } else {
                tau = tau_smag;
                if (fallback) ++*fallback;
            }
        }
    }
    if (s->collision == 2) {
        /* HRR: grad[a][b] = d u_a / d x_b of the velocity field (FD part). */
        hrr_equilibrium3(q, rho, u, s->t3norm, feq);
        double Pi[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int i = 0; i < q; ++i) acc += VEL[i][a] * VEL[i][b] * (f[i] - feq[i]);
                double pr = acc + 0.5 * (u[a] * s->F[b] + s->F[a] * u[b]);
                double fd = grad ? -(1.0 / 3.0) * rho * tau * (grad[a][b] + grad[b][a]) : pr;
                Pi[a][b] = s->hrr_sigma * pr + (1.0 - s->hrr_sigma) * fd;
            }
        double f1[27];
        hrr_f1(q, Pi, u, s->t3norm, f1);
        for (int i = 0; i < q; ++i) fstar[i] = feq[i] + (1.0 - 1.0 / tau) * f1[i] + 0.5 * S[i];
        if (u_out)
            for (int a = 0; a < 3; ++a) u_out[a] = u[a];
        if (tau_out) *tau_out = tau;
        return;
    }
    if (s->collision == 1) {
        /* m_neq = M (f - feq), mS = M S; each moment a changes by           */
        /* -s_a m_neq_a + (1 - s_a / 2) mS_a; back with M^-1.                */
        double rate[8] = {0.0, 1.0, 1.0 / tau, s->mrt_rates[0], s->mrt_rates[1], s->mrt_rates[2],
                          s->mrt_rates[3], s->mrt_rates[4]};
        double dm[27];
        for (int a = 0; a < q; ++a) {
            double mn = 0.0, ms = 0.0;
            for (int i = 0; i < q; ++i) {
                mn += s->Mm[a * q + i] * (f[i] - feq[i]);
                ms += s->Mm[a * q + i] * S[i];
            }
            double r = rate[s->mgroup[a]];
            dm[a] = -r * mn + (1.0 - 0.5 * r) * ms;
        }
        for (int i = 0; i < q; ++i) {
            double acc = 0.0;
            for (int a = 0; a < q; ++a) acc += s->Minv[i * q + a] * dm[a];
            fstar[i] = f[i] + acc;
        }
        if (u_out)
            for (int a = 0; a < 3; ++a) u_out[a] = u[a];
        if (tau_out) *tau_out = tau;
        return;
    }
    double wp = 1.0 / tau;
    double wm = 1.0 / (0.5 + s->magic / (tau - 0.5));
    for (int i = 0; i < q; ++i) {
        int ib = opposite(i);
        double fp = 0.5 * (f[i] + f[ib]), fm = 0.5 * (f[i] - f[ib]);
        double ep = 0.5 * (feq[i] + feq[ib]), em = 0.5 * (feq[i] - feq[ib]);
        double sp = 0.5 * (S[i] + S[ib]), sm = 0.5 * (S[i] - S[ib]);
        fstar[i] = f[i] - wp * (fp - ep) - wm * (fm - em) + (1.0 - 0.5 * wp) * sp + (1.0 - 0.5 * wm) * sm;
    }
    if (u_out)
        for (int a = 0; a < 3; ++a) u_out[a] = u[a];
    if (tau_out) *tau_out = tau;
}

/* Collide a single cell without a simulation (for the invariant tests).    */
void orc_collide(int q, const double *f, double tau, double magic, const double *F, int closure, double cs,
                 double *fstar, double *tau_used)
{
    orc_sim s;
    memset(&s, 0, sizeof s);
    s.q = q;
    s.tau = tau;
    s.magic = magic;
    for (int a = 0; a < 3; ++a) s.F[a] = F[a];
    s.closure = closure;
    s.cs = cs;
    collide_cell(&s, f, 0, fstar, 0, tau_used, 0);
}

/* Collide a single cell with the MRT operator (rates as orc_set_mrt).     */
int orc_collide_mrt(int q, const double *f, double tau, const double *rates, const double *F, int closure,
                    double cs, double *fstar, double *tau_used)
{
    orc_sim s;
    memset(&s, 0, sizeof s);
    s.q = q;
    s.tau = tau;
    s.magic = 0.25;
    for (int a = 0; a < 3; ++a) s.F[a] = F[a];
    s.closure = closure;
    s.cs = cs;
    if (orc_set_mrt(&s, rates) != 0) return -1;
    collide_cell(&s, f, 0, fstar, 0, tau_used, 0);
    return 0;
}

/* Non-equilibrium flux of one cell, packed xx,yy,zz,xy,xz,yz (for tests). */
void orc_noneq_flux(int q, const double *f, const double *F, double *P6)
{
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < q; ++i) {
        rho += f[i];
        for (int a = 0; a < 3; ++a) j[a] += VEL[i][a] * f[i];
    }
    double u[3], feq[27];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / rho;
    orc_equilibrium(q, rho, u, feq);
    static const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k) {
        double acc = 0.0;
        for (int i = 0; i < q; ++i) acc += VEL[i][A[k]] * VEL[i][B[k]] * (f[i] - feq[i]);
        P6[k] = acc + 0.5 * (u[A[k]] * F[B[k]] + F[A[k]] * u[B[k]]);
    }
}

/*
 * Streaming of one post-collision population, Eq. (2), in push form: the
 * value v leaving cell (x,y,z) along c_i lands at the neighbour, or, when the
 * link is cut by a wall, returns to the same cell in the opposite direction:
 *   solid neighbour or no-slip face:  g_opp(i)(x) = v
 *   velocity face (u_w, rho_w):      g_opp(i)(x) = v - 6 w_i rho_w (c_i . u_w)
 *   pressure face (rho_w):           g_opp(i)(x) = -v + 2 w_i rho_w (1 + 9/2 (c_i.u)^2 - 3/2 u.u)
 * (u = this cell's velocity).  A link leaving through several non-periodic
 * faces takes the first of no-slip, velocity, pressure (lowest face index
 * among equals).  Periodic faces wrap.
 * The target cell and slot are returned through tgt/dir.
 */
static double push_target(const orc_sim *s, int x, int y, int z, int i, double v, const double *u, int64_t *tgt,
                          int *dir)
{
    int p[3] = {x + VEL[i][0], y + VEL[i][1], z + VEL[i][2]};
    int ext[3] = {s->nx, s->ny, s->nz};
    int cut_kind = -1, cut_face = -1;
    static const int rank_of[5] = {0, 3, 2, 1, 3}; /* precedence: no-slip (interface) > velocity > pressure */
    for (int a = 0; a < 3; ++a) {
        int face = -1;
        if (p[a] < 0) face = 2 * a;
        if (p[a] >= ext[a]) face = 2 * a + 1;
        if (face < 0) continue;
        if (s->bc[face] == BC_PERIODIC) {
            p[a] = (p[a] + ext[a]) % ext[a];
        } else if (cut_kind < 0 || rank_of[s->bc[face]] > rank_of[cut_kind]) {
            cut_kind = s->bc[face];
            cut_face = face;
        }
    }
    int64_t self = cell_index(s, x, y, z);
    if (cut_kind < 0) {
        int64_t c = cell_index(s, p[0], p[1], p[2]);
        if (!is_solid(s, c)) {
            *tgt = c;
            *dir = i;
            return v;
        }
        cut_kind = BC_NOSLIP;
    }
    *tgt = self;
    *dir = opposite(i);
    double w = weight(s->q, i);
    if (cut_kind == BC_NOSLIP || cut_kind == BC_INTERFACE) return v;
    if (cut_kind == BC_VELOCITY) {
        const double *uw = s->ubc[cut_face];
        double cuw = VEL[i][0] * uw[0] + VEL[i][1] * uw[1] + VEL[i][2] * uw[2];
        return v - 6.0 * w * s->rhobc[cut_face] * cuw;
    }
    double cu = VEL[i][0] * u[0] + VEL[i][1] * u[1] + VEL[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return -v + 2.0 * w * s->rhobc[cut_face] * (1.0 + 4.5 * cu * cu - 1.5 * uu);
}

/*
 * Neighbour of (x,y,z) one cell along axis b in direction dir (+1 or -1),
 * for the finite-difference velocity gradient of HRR:
 *   0  a cell of the domain (fluid; *nb its index, wrapped on periodic axes),
 *   1  a wall half a cell away with velocity uw: a no-slip face (0), a
 *      velocity face (its u_bc) or a solid cell (0),
 *   2  a pressure face: the ghost outside carries the cell's own velocity.
 */
static int fd_neighbour(const orc_sim *s, int x, int y, int z, int b, int dir, int64_t *nb, double *uw)
{
    int p[3] = {x, y, z};
    int ext[3] = {s->nx, s->ny, s->nz};
    p[b] += dir;
    if (p[b] < 0 || p[b] >= ext[b]) {
        int face = 2 * b + (dir > 0);
        if (s->bc[face] == BC_PERIODIC) {
            p[b] = (p[b] + ext[b]) % ext[b];
        } else if (s->bc[face] == BC_PRESSURE) {
            return 2;
        } else {
            for (int a = 0; a < 3; ++a) uw[a] = s->bc[face] == BC_VELOCITY ? s->ubc[face][a] : 0.0;
            return 1;
        }
    }
    int64_t c = cell_index(s, p[0], p[1], p[2]);
    if (is_solid(s, c)) {
        for (int a = 0; a < 3; ++a) uw[a] = 0.0;
        return 1;
    }
    *nb = c;
    return 0;
}

/*
 * Velocity gradient G[a][b] = d u_a / d x_b of the field uf [3][n] at a
 * fluid cell: central differences between two domain neighbours; next to a
 * wall (half a cell away, velocity uw) the derivative of the quadratic
 * through the wall point and the two nearest cells, -4/3 uw + u0 + u1/3
 * (mirrored on the + side); between two walls (uw+ - uw-); a pressure-face
 * ghost takes the cell's own value.  Pinned by exactness on linear and
 * quadratic fields (tests).
 */
static void fd_gradient(const orc_sim *s, const double *uf, int x, int y, int z, double G[3][3])
{
    int64_t N = s->n, c0 = cell_index(s, x, y, z);
    for (int b = 0; b < 3; ++b) {
        int64_t im = -1, ip = -1;
        double wm[3] = {0, 0, 0}, wp[3] = {0, 0, 0};
        int km = fd_neighbour(s, x, y, z, b, -1, &im, wm);
        int kp = fd_neighbour(s, x, y, z, b, +1, &ip, wp);
        for (int a = 0; a < 3; ++a) {
            double u0 = uf[a * N + c0];
            double um = km == 0 ? uf[a * N + im] : u0;
            double up = kp == 0 ? uf[a * N + ip] : u0;
            double d;
            if (km == 1 && kp == 1)
                d = wp[a] - wm[a];
            else if (km == 1)
                d = -(4.0 / 3.0) * wm[a] + u0 + up / 3.0;
            else if (kp == 1)
                d = (4.0 / 3.0) * wp[a] - u0 - um / 3.0;
            else
                d = 0.5 * (up - um);
            G[a][b] = d;
        }
    }
}

/* Gradient of a velocity field at every cell (for the tests): G [9][n],    */
/* row 3a + b = d u_a / d x_b; solid cells get zeros.                       */
void orc_fd_gradient(const orc_sim *s, const double *uf, double *G)
{
    int64_t N = s->n;
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                int64_t c = cell_index(s, x, y, z);
                double g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                if (!is_solid(s, c)) fd_gradient(s, uf, x, y, z, g);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) G[(3 * a + b) * N + c] = g[a][b];
            }
}

/* HRR state: the velocity field u = (j + F/2)/rho of the current populations */
/* (zero at solid cells), the FD gradient's input on the next step.          */
static void hrr_update_velocity(orc_sim *s)
{
    if (s->collision != 2 || !s->uprev || !s->f) return;
    int64_t N = s->n;
    for (int64_t c = 0; c < N; ++c) {
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < s->q; ++i) {
            double v = s->f[i * N + c];
            r += v;
            for (int a = 0; a < 3; ++a) j[a] += VEL[i][a] * v;
        }
        for (int a = 0; a < 3; ++a) s->uprev[a * N + c] = is_solid(s, c) ? 0.0 : (j[a] + 0.5 * s->F[a]) / r;
    }
}

/* Select the HRR collision (D3Q19 only) with the weight sigma in [0, 1] of */
/* the projected flux.  Returns -1 for another stencil or sigma outside.    */
int orc_set_hrr(orc_sim *s, double sigma)
{
    if (s->q != 19 || !(sigma >= 0.0 && sigma <= 1.0)) return -1;
    s->collision = 2;
    s->hrr_sigma = sigma;
    orc_hrr_norms(s->t3norm);
    if (!s->uprev) s->uprev = (double *)calloc((size_t)(3 * s->n), sizeof(double));
    hrr_update_velocity(s);
    return 0;
}

/* One HRR collision of a single cell with a given velocity gradient       */
/* grad[3][3] (row a: d u_a / d x_b), for the invariant tests.             */
void orc_collide_hrr(const double *f, double tau, double sigma, const double *F, const double *grad,
                     double *fstar)
{
    orc_sim s;
    memset(&s, 0, sizeof s);
    s.q = 19;
    s.tau = tau;
    s.magic = 0.25;
    for (int a = 0; a < 3; ++a) s.F[a] = F[a];
    s.collision = 2;
    s.hrr_sigma = sigma;
    orc_hrr_norms(s.t3norm);
    double G[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) G[a][b] = grad[3 * a + b];
    collide_cell(&s, f, (const double(*)[3])G, fstar, 0, 0, 0);
}

/*
 * Advance n time steps: for every fluid cell collide (Eq. 1) and push every
 * population to its destination (Eq. 2) in a second lattice, then swap.
 * Pinned by Poiseuille, Taylor-Green, conservation, symmetry and plug-flow
 * tests.
 */
void orc_step(orc_sim *s, int64_t nsteps)
{
    ensure_lattices(s);
    int q = s->q;
    int64_t N = s->n;
    /* HRR: the gradient of this step uses the velocity field of the previous */
    /* step (uprev); the velocities of this step go to unext                   */
    double *unext = s->collision == 2 ? (double *)calloc((size_t)(3 * N), sizeof(double)) : 0;
    for (int64_t t = 0; t < nsteps; ++t) {
        int64_t fb = 0;
#pragma omp parallel for schedule(static) reduction(+ : fb)
        for (int z = 0; z < s->nz; ++z)
            for (int y = 0; y < s->ny; ++y)
                for (int x = 0; x < s->nx; ++x) {
                    int64_t c = cell_index(s, x, y, z);
                    if (is_solid(s, c)) continue;
                    double f[27], fs[27], u[3], G[3][3];
                    for (int i = 0; i < q; ++i) f[i] = s->f[i * N + c];
                    if (unext) fd_gradient(s, s->uprev, x, y, z, G);
                    collide_cell(s, f, unext ? (const double(*)[3])G : 0, fs, u, 0, &fb);
                    if (unext)
                        for (int a = 0; a < 3; ++a) unext[a * N + c] = u[a];
                    for (int i = 0; i < q; ++i) {
                        int64_t tgt;
                        int d;
                        double v = push_target(s, x, y, z, i, fs[i], u, &tgt, &d);
                        s->g[d * N + tgt] = v;
                    }
                }
        s->fallbacks += fb;
        double *tmp = s->f;
        s->f = s->g;
        s->g = tmp;
        if (unext) {
            tmp = s->uprev;
            s->uprev = unext;
            unext = tmp;
        }
    }
    free(unext);
}

/* ------------------------------------------------------------------------ */
/* 2:1 grid refinement (the block forest's 2:1 refinement, Section 3; the     */
/* coarse-to-fine and fine-to-coarse kernels of the LAGOON runs, Section 5.2). */
/* The paper gives no algorithm; this is the mass-conservative volumetric     */
/* scheme of Rohde, Kandhai, Derksen & van den Akker (2006): coarse packets   */
/* spread evenly over the fine cells they enter ("explosion"), fine packets   */
/* summed into the coarse cell they enter ("coalescence").                   */
/* A coarse lattice and fine lattices below (its -y face) and/or above (its   */
/* +y face), each fine lattice twice as fine in every direction (nx, nz       */
/* twice the coarse ones, x and z periodic on every level), the fine         */
/* relaxation time 1/2 + 2 (tau_c - 1/2) and force F_c / 2 (acoustic         */
/* scaling: the same viscosity and acceleration in physical units).  The      */
/* faces between the levels are BC_INTERFACE faces: within a lattice they     */
/* return each population into the emitting cell (as no-slip faces do), and   */
/* the packets that crossed are exchanged between steps, populations read as  */
/* mass densities (a fine cell holds 1/8 of a coarse cell's volume):          */
/*   coarse to fine: the packet f*_i a coarse interface cell X sends across   */
/*     in coarse step t -> t+1 (canonical f_opp(i)(X) after that step)        */
/*     enters the fine level over both fine substeps: after each substep,    */
/*     every fine interface cell whose source point x_f - c_i (fine units)    */
/*     lies in X takes it as its population i (four fine cells per substep:   */
/*     mass 2 x 4 x f / 8 = f).  The first substep of the next coarse step    */
/*     therefore collides the second half of this step's packets.             */
/*   fine to coarse: the packets f*_i the fine interface cells send across in  */
/*     the two substeps (canonical f_opp(i)(x_f) after each) are summed over  */
/*     the fine cells whose target point x_f + c_i lies in coarse cell Y,     */
/*     divided by 8, and arrive in Y as its population i at t+1.              */
/* Order per coarse step: coarse step; record the coarse packets; twice: fine  */
/* step, add the fine packets, fine interface row from the recorded packets;   */
/* coarse interface row from the sums.  Between steps every slot holds mass  */
/* that belongs to its level, so M_c + M_f / 8 is conserved exactly.  The     */
/* even spreading makes the interface first-order accurate (the levels are    */
/* second order); force-driven channel flow across it stays exact.            */
/* Interface rows hold no solid cells; TRT or MRT (same ghost rates), no       */
/* closure, no HRR.  Pinned by a brute-force emulation of the exchange, exact  */
/* mass conservation, invariance of a uniform moving state, the exact         */
/* force-driven channel across both interfaces and first-order convergence   */
/* to a run that is fine everywhere (tests).                                  */
/* ------------------------------------------------------------------------ */
static int64_t wrapi(int64_t v, int64_t n) { return ((v % n) + n) % n; }

/* Refinement geometry check; returns 0 if coarse/fine fit (fine on side     */
/* `above` of the coarse lattice).                                           */
static int refine_pair_ok(const orc_sim *c, const orc_sim *f, int above)
{
    if (!f) return 0;
    if (f->q != c->q || f->nx != 2 * c->nx || f->nz != 2 * c->nz) return -1;
    if (c->bc[0] != BC_PERIODIC || c->bc[4] != BC_PERIODIC || f->bc[0] != BC_PERIODIC || f->bc[4] != BC_PERIODIC)
        return -1;
    if (c->bc[above ? 3 : 2] != BC_INTERFACE || f->bc[above ? 2 : 3] != BC_INTERFACE) return -1;
    if (fabs(f->tau - (0.5 + 2.0 * (c->tau - 0.5))) > 1e-12 * c->tau) return -1;
    /* TRT or MRT (same ghost rates) without a closure: HRR's gradient would  */
    /* span the levels, and a closure's scaling between levels is not defined */
    if (c->collision != f->collision || c->collision == 2 || c->closure || f->closure) return -1;
    if (c->collision == 1)
        for (int k = 0; k < 5; ++k)
            if (c->mrt_rates[k] != f->mrt_rates[k]) return -1;
    if (c->magic != f->magic) return -1;
    int yc = above ? c->ny - 1 : 0, yf = above ? 0 : f->ny - 1;
    for (int z = 0; z < c->nz; ++z)
        for (int x = 0; x < c->nx; ++x)
            if (is_solid(c, cell_index(c, x, yc, z))) return -1;
    for (int z = 0; z < f->nz; ++z)
        for (int x = 0; x < f->nx; ++x)
            if (is_solid(f, cell_index(f, x, yf, z))) return -1;
    for (int a = 0; a < 3; ++a)
        if (fabs(f->F[a] - 0.5 * c->F[a]) > 1e-15 + 1e-12 * fabs(c->F[a])) return -1;
    return 0;
}

/* One interface: coarse row yc of the coarse lattice, fine row yf of the    */
/* fine lattice; dy = +1 if the fine lattice lies above (coarse packets      */
/* toward the fine level have c_y = dy).  cout, acc: [q][nzc][nxc].          */
static void refine_record_coarse(const orc_sim *c, int yc, int dy, double *cout)
{
    int64_t N = c->n, plane = (int64_t)c->nx * c->nz;
    for (int i = 0; i < c->q; ++i) {
        if (VEL[i][1] != dy) continue;
        for (int z = 0; z < c->nz; ++z)
            for (int x = 0; x < c->nx; ++x)
                cout[i * plane + (int64_t)z * c->nx + x] = c->f[opposite(i) * N + cell_index(c, x, yc, z)];
    }
}

/* Fine interface row after a fine substep: fine cell x_f takes, as its     */
/* population j, the packet of the coarse cell containing its source point   */
/* x_f - c_j (fine units).                                                   */
static void refine_fill_fine(orc_sim *f, const orc_sim *c, int yf, int dy, const double *cout)
{
    int64_t N = f->n, plane = (int64_t)c->nx * c->nz;
    for (int j = 0; j < f->q; ++j) {
        if (VEL[j][1] != dy) continue;
        for (int z = 0; z < f->nz; ++z)
            for (int x = 0; x < f->nx; ++x) {
                int64_t px = wrapi(x - VEL[j][0], f->nx) / 2, pz = wrapi(z - VEL[j][2], f->nz) / 2;
                f->f[j * N + cell_index(f, x, yf, z)] = cout[j * plane + pz * c->nx + px];
            }
    }
}

/* Fine packets sent across in a substep: 1/8 of each goes to the coarse     */
/* cell containing the target point x_f + c_i (fine units); the first       */
/* substep clears the sums.                                                 */
static void refine_add_fine(const orc_sim *f, const orc_sim *c, int yf, int dy, double *acc, int first)
{
    int64_t N = f->n, plane = (int64_t)c->nx * c->nz;
    for (int i = 0; i < f->q; ++i) {
        if (VEL[i][1] != -dy) continue;
        if (first)
            for (int64_t k = 0; k < plane; ++k) acc[i * plane + k] = 0.0;
        for (int z = 0; z < f->nz; ++z)
            for (int x = 0; x < f->nx; ++x) {
                int64_t yx = wrapi(x + VEL[i][0], f->nx) / 2, yz = wrapi(z + VEL[i][2], f->nz) / 2;
                acc[i * plane + yz * c->nx + yx] += f->f[opposite(i) * N + cell_index(f, x, yf, z)] / 8.0;
            }
    }
}

static void refine_fill_coarse(orc_sim *c, int yc, int dy, const double *acc)
{
    int64_t N = c->n, plane = (int64_t)c->nx * c->nz;
    for (int i = 0; i < c->q; ++i) {
        if (VEL[i][1] != -dy) continue;
        for (int z = 0; z < c->nz; ++z)
            for (int x = 0; x < c->nx; ++x)
                c->f[i * N + cell_index(c, x, yc, z)] = acc[i * plane + (int64_t)z * c->nx + x];
    }
}

/* A hierarchy of levels (the paper's block forest refines 2:1 level by      */
/* level, Section 3; the LAGOON runs use ten levels, Section 5.2): node k is  */
/* lattice sims[k] with finer lattices lo[k] below and hi[k] above it (node   */
/* indices, -1 for none), children after their parent, node 0 the coarsest.  */
/* Advancing a node one step: its lattice takes one step; for each child, the */
/* packets crossing into it are recorded and, twice, the child advances one   */
/* step (recursively, its own children included), its packets are added and  */
/* its interface row takes the recorded packets; then the node's interface    */
/* rows take the sums.  Each pair of levels exchanges as stated above, and    */
/* sum over levels of M_level / 8^level is conserved exactly.                 */
typedef struct {
    orc_sim **sims;
    const int *lo, *hi;
    double **buf; /* per node: [2 sides][cout, acc][q][nz][nx] or NULL */
} refine_tree;

static void refine_advance(const refine_tree *T, int k)
{
    orc_sim *c = T->sims[k];
    int child[2] = {T->lo[k], T->hi[k]};
    int64_t plane = (int64_t)c->nx * c->nz;
    orc_step(c, 1);
    for (int side = 0; side < 2; ++side) {
        if (child[side] < 0) continue;
        orc_sim *f = T->sims[child[side]];
        int dy = side ? 1 : -1, yc = side ? c->ny - 1 : 0, yf = side ? 0 : f->ny - 1;
        double *cout = T->buf[k] + (int64_t)(2 * side) * c->q * plane, *acc = cout + (int64_t)c->q * plane;
        refine_record_coarse(c, yc, dy, cout);
        for (int sub = 0; sub < 2; ++sub) {
            refine_advance(T, child[side]);
            refine_add_fine(f, c, yf, dy, acc, sub == 0);
            refine_fill_fine(f, c, yf, dy, cout);
        }
    }
    for (int side = 0; side < 2; ++side) {
        if (child[side] < 0) continue;
        int dy = side ? 1 : -1, yc = side ? c->ny - 1 : 0;
        refine_fill_coarse(c, yc, dy, T->buf[k] + (int64_t)(2 * side + 1) * c->q * plane);
    }
}

/* Advance the hierarchy n steps of node 0 (a node at depth d takes 2^d n   */
/* steps).  Returns -1 if the nodes do not form a refinement tree: a child   */
/* index not after its parent, a node with two parents or none (except node */
/* 0), an interface face without a child or a child without an interface    */
/* face, or a parent/child pair that does not fit (refine_pair_ok); or if a */
/* buffer cannot be allocated.                                              */
int orc_refine_tree_step(orc_sim **sims, const int *lo, const int *hi, int count, int64_t n)
{
    if (count < 1 || count > 4096) return -1;
    int *parents = (int *)calloc((size_t)count, sizeof(int));
    int *up = (int *)calloc((size_t)count, sizeof(int)); /* face index toward the parent, 0 for none */
    double **buf = (double **)calloc((size_t)count, sizeof(double *));
    int bad = !parents || !up || !buf;
    for (int k = 0; k < count && !bad; ++k) {
        int child[2] = {lo[k], hi[k]};
        if (!sims[k]) bad = 1;
        for (int side = 0; side < 2 && !bad; ++side) {
            if (child[side] < 0) continue;
            if (child[side] <= k || child[side] >= count || !sims[child[side]]) { bad = 1; break; }
            parents[child[side]]++;
            up[child[side]] = side ? 2 : 3; /* a lower child meets its parent with its +y face */
            if (refine_pair_ok(sims[k], sims[child[side]], side)) bad = 1;
        }
    }
    for (int k = 1; k < count && !bad; ++k)
        if (parents[k] != 1) bad = 1;
    /* a y face is an interface exactly where it leads to a child or faces the parent */
    for (int k = 0; k < count && !bad; ++k) {
        int child[2] = {lo[k], hi[k]};
        for (int side = 0; side < 2 && !bad; ++side) {
            int face = side ? 3 : 2, has = child[side] >= 0, toward = up[k] == face;
            if (has && toward) bad = 1;
            else if ((sims[k]->bc[face] == BC_INTERFACE) != (has || toward)) bad = 1;
        }
    }
    for (int k = 0; k < count && !bad; ++k) {
        ensure_lattices(sims[k]);
        if (lo[k] >= 0 || hi[k] >= 0) {
            buf[k] = (double *)calloc((size_t)(4 * sims[k]->q * (int64_t)sims[k]->nx * sims[k]->nz), sizeof(double));
            if (!buf[k]) bad = 1;
        }
    }
    if (!bad) {
        refine_tree T = {sims, lo, hi, buf};
        for (int64_t t = 0; t < n; ++t) refine_advance(&T, 0);
    }
    if (buf)
        for (int k = 0; k < count; ++k) free(buf[k]);
    free(buf);
    free(up);
    free(parents);
    return bad ? -1 : 0;
}

/* Two levels: the coarse lattice n steps and each fine lattice (nullable)  */
/* 2n steps.  Returns -1 if the lattices do not form a refinement (or the   */
/* exchange buffer cannot be allocated).                                    */
int orc_refine_step(orc_sim *c, orc_sim *fine_lo, orc_sim *fine_hi, int64_t n)
{
    orc_sim *sims[3] = {c, 0, 0};
    int lo[3] = {-1, -1, -1}, hi[3] = {-1, -1, -1}, count = 1;
    if (fine_lo) {
        sims[count] = fine_lo;
        lo[0] = count++;
    }
    if (fine_hi) {
        sims[count] = fine_hi;
        hi[0] = count++;
    }
    return orc_refine_tree_step(sims, lo, hi, count, n);
}

/* Density and velocity u = (j + F/2)/rho of the canonical state; u [3][n]. */
void orc_moments(orc_sim *s, double *rho, double *u)
{
    ensure_lattices(s);
    int64_t N = s->n;
    for (int64_t c = 0; c < N; ++c) {
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < s->q; ++i) {
            double v = s->f[i * N + c];
            r += v;
            for (int a = 0; a < 3; ++a) j[a] += VEL[i][a] * v;
        }
        rho[c] = r;
        for (int a = 0; a < 3; ++a) u[a * N + c] = is_solid(s, c) ? 0.0 : (j[a] + 0.5 * s->F[a]) / r;
    }
}

/* Totals over fluid cells: mass = sum rho, mom = sum j (raw first moment). */
void orc_totals(orc_sim *s, double *mass, double *mom)
{
    ensure_lattices(s);
    int64_t N = s->n;
    double m = 0.0, p[3] = {0, 0, 0};
    for (int64_t c = 0; c < N; ++c) {
        if (is_solid(s, c)) continue;
        for (int i = 0; i < s->q; ++i) {
            double v = s->f[i * N + c];
            m += v;
            for (int a = 0; a < 3; ++a) p[a] += VEL[i][a] * v;
        }
    }
    *mass = m;
    for (int a = 0; a < 3; ++a) mom[a] = p[a];
}

/*
 * Probe: canonical populations at selected cells after k steps, starting
 * from f^eq(rho, u) of the given fields (t = 0), without storing a lattice.
 * Each value at (y, i, t+1) is the single push of Eq. (2) that lands there:
 * from y - c_i when that cell is a fluid cell reached without crossing a
 * non-periodic face, else from y itself in direction opposite(i) (the cut
 * link).  Recursion depth k; cost grows as Q^k per probed cell, so keep k
 * small (1..3).  out[ncell][q].
 * Pinned against orc_step on small domains (tests).
 */
static void probe_rec(const orc_sim *s, const double *rho, const double *u, int x, int y, int z, int k,
                      double *f_out);

static void probe_post(const orc_sim *s, const double *rho, const double *u, int x, int y, int z, int k,
                       double *fs, double *uc)
{
    double f[27];
    probe_rec(s, rho, u, x, y, z, k, f);
    collide_cell(s, f, 0, fs, uc, 0, 0);
}

static void probe_rec(const orc_sim *s, const double *rho, const double *u, int x, int y, int z, int k,
                      double *f_out)
{
    int64_t c = cell_index(s, x, y, z);
    if (k == 0) {
        double uc[3] = {u[c], u[s->n + c], u[2 * s->n + c]};
        orc_equilibrium(s->q, rho[c], uc, f_out);
        return;
    }
    int ext[3] = {s->nx, s->ny, s->nz};
    for (int i = 0; i < s->q; ++i) {
        int p[3] = {x - VEL[i][0], y - VEL[i][1], z - VEL[i][2]};
        int crossed = 0;
        for (int a = 0; a < 3; ++a) {
            if (p[a] >= 0 && p[a] < ext[a]) continue;
            int face = p[a] < 0 ? 2 * a : 2 * a + 1;
            if (s->bc[face] == BC_PERIODIC)
                p[a] = (p[a] + ext[a]) % ext[a];
            else
                crossed = 1;
        }
        int64_t tgt;
        int d;
        double fs[27], uc[3], v;
        if (!crossed && !is_solid(s, cell_index(s, p[0], p[1], p[2]))) {
            probe_post(s, rho, u, p[0], p[1], p[2], k - 1, fs, uc);
            v = push_target(s, p[0], p[1], p[2], i, fs[i], uc, &tgt, &d);
        } else {
            probe_post(s, rho, u, x, y, z, k - 1, fs, uc);
            v = push_target(s, x, y, z, opposite(i), fs[opposite(i)], uc, &tgt, &d);
        }
        f_out[i] = (tgt == c && d == i) ? v : NAN;
    }
}

void orc_probe(const orc_sim *s, const double *rho, const double *u, int k, int64_t ncell, const int64_t *cells,
               double *out)
{
    if (s->collision == 2) { /* HRR's gradient depends on the step history: no probe */
        for (int64_t r = 0; r < ncell * s->q; ++r) out[r] = NAN;
        return;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < ncell; ++r) {
        int64_t c = cells[r];
        int x = (int)(c % s->nx);
        int y = (int)((c / s->nx) % s->ny);
        int z = (int)(c / ((int64_t)s->nx * s->ny));
        probe_rec(s, rho, u, x, y, z, k, out + r * s->q);
    }
}

/* ------------------------------------------------------------------------ */
/* Training-data builders for the learned closure.                           */
/* ------------------------------------------------------------------------ */

/*
 * Box filter: average fine fields over non-overlapping 4x4x4 blocks.
 * rho[nf], u[3][nf] in; out[10][nc] = rho, u_x, u_y, u_z, then the filtered
 * products uu in the order xx, yy, zz, xy, xz, yz.  Fine dims must be
 * multiples of 4.  Pinned by: constants map to constants, block sums are
 * preserved, a linear field maps to its block-centre value (tests).
 */
void orc_box_filter4(int nx, int ny, int nz, const double *rho, const double *u, double *out)
{
    int cx = nx / 4, cy = ny / 4, cz = nz / 4;
    int64_t nf = (int64_t)nx * ny * nz, nc = (int64_t)cx * cy * cz;
    static const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
    for (int64_t k = 0; k < 10 * nc; ++k) out[k] = 0.0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t f = ((int64_t)z * ny + y) * nx + x;
                int64_t c = ((int64_t)(z / 4) * cy + y / 4) * cx + x / 4;
                out[c] += rho[f] / 64.0;
                for (int a = 0; a < 3; ++a) out[(1 + a) * nc + c] += u[a * nf + f] / 64.0;
                for (int m = 0; m < 6; ++m) out[(4 + m) * nc + c] += u[A[m] * nf + f] * u[B[m] * nf + f] / 64.0;
            }
}

/*
 * Derivative of a cell-centred field g along axis a at cell index i (0..n-1):
 * central difference inside; on a periodic axis the stencil wraps; next to a
 * wall face (non-periodic axis, wall halfway outside the first/last cell,
 * value zero there) the derivative of the quadratic through the wall point
 * and the two nearest cells: d = g0 + g1/3 at the low wall, mirrored at the
 * high wall.  Pinned by exactness on quadratics (tests).
 */
static double deriv(const double *g, int64_t stride, int i, int n, int periodic)
{
    if (periodic) {
        int im = (i - 1 + n) % n, ip = (i + 1) % n;
        return 0.5 * (g[(int64_t)ip * stride] - g[(int64_t)im * stride]);
    }
    if (n == 1) return 0.0;
    if (i == 0) return g[0] + g[stride] / 3.0;
    if (i == n - 1) return -(g[(int64_t)(n - 1) * stride] + g[(int64_t)(n - 2) * stride] / 3.0);
    return 0.5 * (g[(int64_t)(i + 1) * stride] - g[(int64_t)(i - 1) * stride]);
}

/* Filtered strain rate S (packed xx,yy,zz,xy,xz,yz) of the coarse field u. */
void orc_strain(int cx, int cy, int cz, const int *periodic, const double *u, double *S)
{
    int64_t nc = (int64_t)cx * cy * cz;
    int ext[3] = {cx, cy, cz};
    int64_t strd[3] = {1, cx, (int64_t)cx * cy};
    for (int z = 0; z < cz; ++z)
        for (int y = 0; y < cy; ++y)
            for (int x = 0; x < cx; ++x) {
                int64_t c = ((int64_t)z * cy + y) * cx + x;
                int pos[3] = {x, y, z};
                double G[3][3]; /* G[a][b] = d u_a / d x_b */
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        const double *base = u + a * nc + c - (int64_t)pos[b] * strd[b];
                        G[a][b] = deriv(base, strd[b], pos[b], ext[b], periodic[b]);
                    }
                S[0 * nc + c] = G[0][0];
                S[1 * nc + c] = G[1][1];
                S[2 * nc + c] = G[2][2];
                S[3 * nc + c] = 0.5 * (G[0][1] + G[1][0]);
                S[4 * nc + c] = 0.5 * (G[0][2] + G[2][0]);
                S[5 * nc + c] = 0.5 * (G[1][2] + G[2][1]);
            }
}

/*
 * Closure dataset from box-filtered fields filt[10][nc] (as produced by
 * orc_box_filter4): per coarse cell the target dtau* = 3 nu_t* with
 *   tau_sgs = <u u> - <u><u>,  nu_t* = max(0, -dev(tau_sgs):S / (2 S:S + eps)),
 * and the six features of the flux the coarse lattice would carry,
 * P = -(2/3)(tau + dtau*) S.  x[nc][6], t[nc].
 * Pinned by the closed form of a box-filtered linear fine field (subgrid
 * stress 1.25 G G^T, strain 4 sym G, target and features), which a dropped
 * dev, a wrong contraction weight, sign, factor or clip fails, and by a
 * pure-shear sample (tests).
 */
void orc_closure_dataset(int cx, int cy, int cz, const int *periodic, const double *filt, double tau, double cs,
                         double eps, double *x, double *t)
{
    int64_t nc = (int64_t)cx * cy * cz;
    double *S = (double *)malloc(sizeof(double) * 6 * nc);
    orc_strain(cx, cy, cz, periodic, filt + nc, S);
    static const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
    for (int64_t c = 0; c < nc; ++c) {
        double ts[6], Sc[6];
        for (int m = 0; m < 6; ++m) {
            ts[m] = filt[(4 + m) * nc + c] - filt[(1 + A[m]) * nc + c] * filt[(1 + B[m]) * nc + c];
            Sc[m] = S[m * nc + c];
        }
        double trt = (ts[0] + ts[1] + ts[2]) / 3.0;
        double dd = 0.0, ss = 0.0;
        for (int m = 0; m < 6; ++m) {
            double mult = m < 3 ? 1.0 : 2.0;
            double tdev = m < 3 ? ts[m] - trt : ts[m];
            dd += mult * tdev * Sc[m];
            ss += mult * Sc[m] * Sc[m];
        }
        double nut = -dd / (2.0 * ss + eps);
        if (nut < 0.0) nut = 0.0;
        double dtau = 3.0 * nut;
        double P[6];
        for (int m = 0; m < 6; ++m) P[m] = -(2.0 / 3.0) * (tau + dtau) * Sc[m];
        orc_features(P, filt[c], tau, cs, x + 6 * c);
        t[c] = dtau;
    }
    free(S);
}

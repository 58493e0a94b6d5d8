/*
 * rbsog.h -- C-ABI of the MI355X (gfx950) library for the random batch
 * sum-of-Gaussians (RBSOG) force evaluation and velocity-Verlet step of 3-D
 * periodic Yukawa systems (Chen, Liang & Xu, "Random batch sum-of-Gaussians
 * algorithm for molecular dynamics simulations of Yukawa systems in three
 * dimensions").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an int status: RBSOG_OK (0) or a negative code;
 *    rbsog_last_error() returns a thread-local message for the last failure.
 *    Nothing throws across this interface.
 *  - Pointers named *_dev are device pointers (HIP global memory on the GPU the
 *    handle was created on); pointers named *_host, and struct pointers, are
 *    host pointers.  The caller owns every buffer it passes.
 *  - Particle arrays are FP64 structure-of-arrays in the caller's particle
 *    order: x[3*N] = {x_0..x_{N-1}, y_0..y_{N-1}, z_0..z_{N-1}}, likewise v and
 *    f; q[N] charges, m[N] masses.  Positions lie in the cubic box [0, L)^3.
 *  - All device work is enqueued on the HIP stream given at creation (passed
 *    as void* so this header needs no HIP include) and is asynchronous with
 *    respect to the host unless a function says otherwise.
 *  - The single-system path allocates no device memory after rbsog_create:
 *    every scratch buffer lives in the caller's workspace, sized by
 *    rbsog_workspace_size.
 *  - Force-evaluation index: the random Fourier modes of an evaluation are a
 *    pure function of (seed, replica, step), so any evaluation can be repeated
 *    or resumed.  rbsog_step uses step0 for the force given on entry and
 *    step0 + n + 1 for the force after the (n+1)-th drift.
 */
#ifndef RBSOG_H
#define RBSOG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define RBSOG_OK 0
#define RBSOG_EINVAL (-1)      /* invalid argument or parameter combination */
#define RBSOG_ENOROOT (-2)     /* no C1 starting point with positive weight / no SOG meets eps */
#define RBSOG_EWORKSPACE (-3)  /* workspace missing, misaligned or too small */
#define RBSOG_EAGAIN (-4)      /* served ensemble: no slot or memory free now */
#define RBSOG_ENONFINITE (-5)  /* a non-finite force or position was produced */
#define RBSOG_EHIP (-6)        /* a HIP runtime call failed */
#define RBSOG_ENOMEM (-7)      /* host memory allocation failed */

/* precision of the force arithmetic */
#define RBSOG_FP64 0   /* everything in FP64 */
#define RBSOG_MIXED 1  /* pair-kernel and per-particle phase arithmetic in FP32;
                          positions, k.r argument reduction, rho(k) and force
                          accumulation, integration and energies in FP64 */

/* correction F(k) of the importance-sampling measure P(k) = F(k) Fhat(k) / S
 * (Section 4.3, eq. 3.124) */
#define RBSOG_ADAPTIVE 0  /* Debye-Hueckel leading term of eq. (3.22), as printed:
                             kTV / (kTV / sum q^2 + lambda^2 / (1 + lambda^2 k^2)) */
#define RBSOG_FLAT 1      /* F = 1 (the density of the random batch Ewald method) */
#define RBSOG_K2 2        /* F = k^2 (the density of the earlier Coulomb RBSOG) */
#define RBSOG_DH4PI 3     /* as ADAPTIVE with 4 pi lambda^2 in place of lambda^2 */

#define RBSOG_AUTO (-999)   /* M1 = M2 = RBSOG_AUTO: choose the numbers of Gaussians */
#define RBSOG_MAX_GAUSS 32
/* Doubles in one energy row (rbsog_compute_forces, rbsog_step, rbsog_ens_retire). */
#define RBSOG_ENERGY_COLS 8

/*
 * SOG decomposition Y(r) = N(r) + F(r) of the Yukawa kernel
 * Y(r) = exp(-r/lambda)/r (Section 3, Algorithm 1, C1-continuous form):
 *   F(r)    = h [ w f(t_{M2}, r) + sum_{m=-M1}^{M2-1} f(t_m, r) ]  (eq. 2.41;
 *             with smooth = 2 the m = M2 term has exponent e^{t_M2} sigma r^2, eq. c2)
 *           = sum_j c[j] exp(-s[j] r^2),     j = m + M1, m = -M1..M2,
 *   Fhat(k) = sum_j A[j] exp(-B[j] k^2)      (its 3-D Fourier transform, Section 4.1),
 * with f(t,r) = pi^{-1/2} exp(-r^2 e^t - e^{-t}/(4 lambda^2) + t/2) (eq. ftr),
 * t_m = t0 + m h, and N(r) = Y(r) - F(r) for r < r_c, 0 beyond (eq. short).
 */
typedef struct rbsog_sog {
    double lambda, r_c, eps; /* inputs: screening length, near cutoff, tolerance   */
    double h, t0, w;         /* step (eq. 2.30), starting point, weight of m = M2  */
    int M1, M2, n;           /* n = M1 + M2 + 1 Gaussians (1..RBSOG_MAX_GAUSS)     */
    double c[RBSOG_MAX_GAUSS], s[RBSOG_MAX_GAUSS];
    double A[RBSOG_MAX_GAUSS], B[RBSOG_MAX_GAUSS];
    double F0;               /* F(0) = sum c                                         */
    double Fhat0;            /* Fhat(0) = sum A                                      */
    double max_err;          /* max |Y - F| on [r_c, 33 lambda] (sampled densely)    */
    int smooth;              /* 2: the C2 form of Appendix C (sigma used); else C1   */
    double sigma;            /* C2: the narrowest Gaussian's exponent is e^{t_M2} sigma */
    /* The kernel (zero-initialised: the Yukawa kernel above).  nyuk = 2: the
     * exact gradient-corrected screening kernel of Section 1,
     * Y(r) = ya[0] e^{-r/yl[0]}/r + ya[1] e^{-r/yl[1]}/r (rbsog_sog_init_egs);
     * then c, s, A, B hold both terms' Gaussians (n of them), and h, t0, w,
     * M1, M2, sigma are those of the first term's decomposition.            */
    int nyuk;                /* 0 or 1: Yukawa; 2: the EGS kernel               */
    double nu;               /* EGS gradient-correction strength, 0 < nu < 1     */
    double ya[2], yl[2];     /* nyuk = 2: weights and lengths of the two terms   */
} rbsog_sog;

/*
 * Algorithm 1 (Section 3.2): h from eq. (2.30) with delta = r_c, then
 * smooth = 1: the smallest starting point t0 in [0, h) that makes the
 *   decomposition C1 at r_c (eq. 1.25) with w from the C0 condition
 *   (eq. 2.42) and w > 0;
 * smooth = 2 (Appendix C, eq. c2): the narrowest Gaussian also gets a
 *   bandwidth factor sigma, and (t0, w, sigma) make Y - F vanish at r_c with
 *   its first and second derivatives: for each t0 the first two conditions
 *   give sigma and w in closed form and the curvature condition is solved in
 *   t0 (smallest root in [0, h) with w > 0 and sigma > e^{-h}, so that the
 *   adjusted Gaussian stays the narrowest).
 * With M1 = M2 = RBSOG_AUTO the smallest total M1 + M2 + 1 whose error on
 * [r_c, 33 lambda] is <= eps is chosen (for each total, M2 = -12 upward);
 * otherwise the given M1 >= 0, M2 are used.  Host only, no GPU needed.
 * Errors: RBSOG_EINVAL (lambda, r_c or eps not positive and finite,
 * r_c >= 33 lambda, eps >= 1, smooth not 1 or 2, bad M1/M2), RBSOG_ENOROOT.
 */
int rbsog_sog_init(double lambda, double r_c, double eps, int smooth, int M1, int M2, rbsog_sog *out);

/*
 * The exact gradient-corrected screening (EGS) kernel of Section 1, whose
 * dielectric is eps(k) = 1 + (lambda k)^{-2} (1 + nu lambda^2 k^2 / 4)^{-1},
 * as the difference of two Yukawa kernels (partial fractions of
 * 4 pi / (k^2 eps(k))): ya[j] e^{-r/yl[j]}/r with yl[j] = alpha_j^{-1/2},
 * alpha_1 = 2 / (lambda^2 (1 + sqrt(1 - nu))), alpha_2 = 2 (1 + sqrt(1 - nu)) /
 * (nu lambda^2), ya[0] = alpha_2 / (alpha_2 - alpha_1) = 1 - ya[1].  Each term
 * gets the decomposition of rbsog_sog_init (numbers of Gaussians chosen
 * automatically, C1 or C2 as smooth says) at length yl[j] and tolerance
 * eps / (|ya[0]| + |ya[1]|); F is the sum of ya[j] times each term's
 * Gaussians, so |Y - F| <= eps on [r_c, 33 yl[0]] (max_err) and N = Y - F is
 * as smooth at r_c as each term.  A term with r_c >= 33 yl[j] has no Gaussians
 * and lies wholly inside the near field (it is below e^{-33}/r_c at r_c).
 * Systems built on the result use the kernel everywhere: the pair function,
 * the adaptive density of eq. (3.22) (with eps(k)^{-1}/k^2 of this
 * dielectric) and the energy constants.  Host only.
 * Errors: RBSOG_EINVAL (lambda, r_c or eps as rbsog_sog_init, nu outside
 * (0, 1), r_c >= 33 yl[0], more than RBSOG_MAX_GAUSS Gaussians in all),
 * RBSOG_ENOROOT.
 */
int rbsog_sog_init_egs(double lambda, double nu, double r_c, double eps, int smooth, rbsog_sog *out);

/*
 * Recomputes c, s, A, B, F0, Fhat0 and max_err of *sog from its lambda, r_c,
 * h, t0, w, M1, M2 (for a decomposition given by its parameters, e.g. a row of
 * the paper's Table 1).  The expansion is evaluated in a fixed IEEE FP64
 * expression order (t = t0 + m h; s = exp(t);
 * c = (h/sqrt(pi)) exp(t/2 - exp(-t)/(4 lambda^2)) [* w at m = M2];
 * A = pi sqrt(pi) c / (s sqrt(s)); B = 1/(4 s)), so identical parameters give
 * identical coefficients on any conforming host.  Host only.
 * Errors: RBSOG_EINVAL (also for a two-term kernel, nyuk = 2, whose Gaussians
 * come from rbsog_sog_init_egs or the caller).
 */
int rbsog_sog_expand(rbsog_sog *sog);

/*
 * The near-field pair function, eq. (3.8), as the FP64 kernels evaluate it:
 * H(r) = r^3 [F_N1(r) + F_N2(r)] = exp(-r/lambda)(1 + r/lambda) - r^3 G(r^2)
 * with G(r^2) = sum_m 2 c_m s_m exp(-s_m r^2) (the pair force is
 * q_i q_j H(r)/r^3 d), and K(r) = r (Y(r) - F(r)) (the pair energy is
 * q_i q_j K(r)/r), on 0 <= r <= r_c as polynomials in y = 2 r / r_c - 1,
 * ascending powers written to h[29] and k[29] (Chebyshev interpolation in
 * extended precision, truncated, converted to powers of y; the powers above
 * the degree are zero).  Returns the lowest degree of 24, 26 and 28 at which
 * both are within 1e-15 (absolute; H(0) = K(0) = 1) over the whole interval
 * with FP64 Horner evaluation (then the FP64 pair kernel uses them), 0 when
 * none is (then it evaluates the exponentials one by one).  Host only.
 * Errors: RBSOG_EINVAL.
 */
int rbsog_sog_near_poly(const rbsog_sog *sog, double *h, double *k);

/* One periodic system. */
typedef struct rbsog_params {
    int64_t N;          /* particles, 1 .. 2^27 - 1                                */
    double L;           /* box edge (the x edge of a cuboid, see Ly, Lz);
                           requires floor(L / r_c) >= 3                       */
    double kT;          /* k_B T entering the adaptive density (eq. 3.22), > 0     */
    int P;              /* random-batch size, 1..4096                              */
    int mmax;           /* Fourier lattice 1 <= |n|^2 <= mmax, k = 2 pi n / L;
                           0 = the largest m with Fhat(k^2) >= 1e-16 Fhat(0)       */
    uint64_t seed;      /* Philox key word 0                                       */
    uint32_t replica;   /* Philox key word 1                                       */
    int precision;      /* RBSOG_FP64 or RBSOG_MIXED                               */
    int density;        /* RBSOG_ADAPTIVE, RBSOG_FLAT, RBSOG_K2 or RBSOG_DH4PI     */
    double skin;        /* neighbour-list skin: lists hold pairs within r_c + skin
                           and rbsog_step rebuilds them only when some particle
                           has moved more than skin/2 since the last build; < 0 =
                           default 0.125 r_c; capped so that L >= 3 (r_c + skin);
                           0 = rebuild every step.  Results do not depend on it
                           beyond rounding (sums taken in another order).
                           Hot systems, whose fastest particles cross skin/2 in a
                           step or two, run fastest with 0 (lists of r_c only):
                           the default drops to 0 -- at an rbsog_step whose dt
                           exceeds every earlier one, or at a served replica's
                           admission -- when sqrt(2 ln(3N + 1) kT / m_min) dt >
                           skin/4, and at an rbsog_step after earlier calls
                           rebuilt the lists at more than half of at least ten
                           steps (systems hotter than kT, such as a random
                           start relaxing); the fine grid and list capacity are
                           then re-derived for lists of r_c (rbsog_get_info
                           reports the new skin, nf and near_capacity). */
    int full_k;         /* 0: random batch of P sampled modes (the method);
                           1: deterministic far field over the whole lattice,
                           coefficient Fhat(k)/V per mode (eqs. 3.5, UF without
                           sampling) -- a test reference, N x nlat work per force;
                           P is then unused and rbsog_compute_rho is refused   */
    int sampler;        /* RBSOG_SAMPLER_IID (0): P i.i.d. modes per step by the
                           inverse CDF of the shell weights;
                           RBSOG_SAMPLER_MH (1): the Metropolis-Hastings chain
                           Section 4.1 names for drawing P(k): an independence
                           chain whose proposals are drawn exactly from the
                           measure with F = 1 (P_q proportional to Fhat) and
                           accepted with probability min(1, F(k')/F(k)); the
                           P modes of a step are the chain's next P states.
                           The chain advances over the modes as the library
                           draws them (ahead, in consecutive steps), so its
                           draws depend on the history of calls as well as on
                           the key; single systems only (not the ensemble)   */
    double Ly, Lz;      /* edges of a cuboid box along y and z (Section 2 and
                           Algorithm 2 take the box as (L_x, L_y, L_z)); 0 =
                           equal to L (a cube).  L is then the x edge; every
                           edge needs floor(L_d / r_c) >= 3.  A cuboid's modes
                           are k = 2 pi (n_x/L_x, n_y/L_y, n_z/L_z) over every
                           n != 0 with Fhat(k^2) >= 1e-16 Fhat(0), ordered by
                           (k^2, n_x, n_y, n_z); its measure (eq. 3.124) is
                           tabled point by point (k^2 no longer groups by
                           |n|^2) and a draw takes the point from one Philox
                           word.  A cuboid requires mmax = 0 and the i.i.d.
                           sampler; the served ensemble, rbsog_ssf and
                           rbsog_rho_noalloc take cubes only.                 */
} rbsog_params;

#define RBSOG_SAMPLER_IID 0
#define RBSOG_SAMPLER_MH 1

typedef struct rbsog_handle rbsog_handle;

/* Derived sizes of a created system (host copy).  skin, nf and near_capacity
 * can change at an rbsog_step when a default skin drops to 0 (see skin). */
typedef struct rbsog_info {
    int64_t N;
    int nc;             /* cells along x, floor(L / r_c)                           */
    int mmax;           /* lattice truncation in use                               */
    int nshell;         /* non-empty shells |n|^2 = m in the lattice               */
    int64_t nlat;       /* lattice points                                          */
    double S;           /* normalisation of P(k) (eq. 3.124)                       */
    double Q1, Q2;      /* sum q, sum q^2                                          */
    size_t ws_bytes;    /* workspace bytes the system needs                        */
    double skin;        /* neighbour-list skin in use                              */
    int nf;             /* cells per axis of the force evaluation's fine grid      */
    int near_capacity;  /* kp: a particle's neighbour list holds up to 5 kp entries */
    int near_poly;      /* degree of the polynomials H, K the FP64 pair kernel uses (0: none; 0 in mixed precision) */
    int nc_y, nc_z;     /* cells along y and z (equal to nc in a cube); the
                           cell list of rbsog_build_cells has nc nc_y nc_z cells,
                           and nshell = nlat in a cuboid (one entry per point) */
} rbsog_info;

/*
 * Bytes of device workspace a system with these parameters needs (the Fourier
 * lattice, sampling tables, cell list, cell-ordered particle copy, sample and
 * structure-factor buffers, reduction partials).  Host only.
 * Errors: RBSOG_EINVAL.
 */
int rbsog_workspace_size(const rbsog_params *p, const rbsog_sog *sog, size_t *bytes);

/*
 * Creates a system.  Builds the Fourier lattice and the shell CDF of P(k) on
 * the host (eq. 3.124 restricted to the lattice; the measure depends on |n|^2
 * only in a cubic box), reads q_dev (to form sum q and sum q^2) and uploads the
 * tables into the caller's workspace, synchronising the stream once.  q_dev and
 * m_dev (N doubles each, device) are referenced, not copied, and must stay
 * valid and unchanged for the handle's lifetime; ws_dev must be 256-byte
 * aligned and at least rbsog_workspace_size bytes, and is owned by the caller.
 * Errors: RBSOG_EINVAL, RBSOG_EWORKSPACE, RBSOG_EHIP, RBSOG_ENOMEM.
 */
int rbsog_create(const rbsog_params *p, const rbsog_sog *sog, const double *q_dev, const double *m_dev,
                 void *ws_dev, size_t ws_bytes, void *hip_stream, rbsog_handle **out);

/* Copies the derived sizes of a system into *out (host).  Errors: RBSOG_EINVAL. */
int rbsog_get_info(const rbsog_handle *h, rbsog_info *out);

/*
 * Cell list of positions x_dev (the neighbour set of eq. 3.8): nc = floor(L/r_c)
 * cells per axis, cell of x is c_d = clamp(floor(x_d nc/L), 0, nc-1),
 * id = (c_z nc + c_y) nc + c_x; particles sorted by id with ties in ascending
 * particle index (a stable sort).  Writes cell_start_dev[nc^3 + 1] and
 * order_dev[N] (int32, device) when non-null; the list is also kept in the
 * workspace.  Errors: RBSOG_EINVAL, RBSOG_EHIP.
 */
int rbsog_build_cells(rbsog_handle *h, const double *x_dev, int32_t *cell_start_dev, int32_t *order_dev);

/*
 * Draws the P Fourier modes of force evaluation `step` from P(k) (Algorithm 2,
 * first step of a time step; eq. 3.124), i.i.d. by inverse CDF:
 *   (w0..w3) = Philox4x64-10(counter = (l, step, 0, 0), key = (seed, replica));
 *   target = ((w0 >> 11) 2^-53) S;  shell = first with cdf > target;
 *   point  = high word of w1 * r3(shell) within the shell, shells sorted by
 *            (|n|^2, nx, ny, nz).
 * Writes n_dev[P][3] (int32 lattice vectors, k = 2 pi n / L) and
 * coef_dev[P] = S / (P V F(k)) (the estimator weight of eq. UF).
 * Errors: RBSOG_EINVAL, RBSOG_EHIP.
 */
int rbsog_sample_k(rbsog_handle *h, uint64_t step, int32_t *n_dev, double *coef_dev);

/*
 * Structure factors rho(k_l) = sum_j q_j exp(i k_l . r_j) (Section 2) of the
 * modes of evaluation `step`, rho_dev[P][2] = (re, im), FP64 accumulation in a
 * fixed order (bitwise reproducible run to run).  Errors: RBSOG_EINVAL, RBSOG_EHIP.
 */
int rbsog_compute_rho(rbsog_handle *h, uint64_t step, const double *x_dev, double *rho_dev);

/*
 * One force evaluation (the force step of Algorithm 2; eq. 3.8 with the random-batch
 * far field of eq. UF):
 *   f_i = sum_{j: |d| < r_c} q_i q_j [F_N1 + F_N2](|d|) d            (near, d = r_i - r_j, minimum image)
 *       - q_i sum_l coef_l k_l Im(exp(-i k_l . r_i) rho(k_l))          (far, random batch)
 * writes f_dev[3*N] (original particle order), f_near_dev[3*N] (nullable) the
 * near part alone, and energy_dev[RBSOG_ENERGY_COLS] (nullable, device) =
 *   { U_N, U*_F, U_k0 = Fhat(0)(sum q)^2/(2V), U_self = -F(0) sum q^2 / 2,
 *     U_bg = -(sum q)^2 4 pi lambda^2/(2V), 0, W_N, W*_F }
 * with the virials W = -3V dU/dV of the near and far parts (configuration
 * scaled with the box, d -> s d, V = L^3):
 *   W_N  = sum over pairs of d . F_ij (N and N' vanish at r_c, the SOG's C0 and
 *          C1 conditions, so pairs at the cutoff add nothing);
 *   W*_F = sum_l coef_l |rho_l|^2 (3/2 - k_l^2 G(k_l^2) / Fhat(k_l^2)),
 *          G = -dFhat/d(k^2) = sum_j A_j B_j exp(-B_j k^2): the random-batch
 *          estimator (the weights of eq. UF) of 3 U_F - (1/V) sum_k k^2 G |rho|^2.
 * U_k0 and U_bg scale as 1/V (virial 3 U_k0 and 3 U_bg), U_self not at all, so
 * the pressure is P = (2 KE + W_N + W*_F + 3 U_k0 + 3 U_bg) / (3V).  All sums
 * in FP64 in both precisions.  Errors: RBSOG_EINVAL, RBSOG_EHIP.
 */
int rbsog_compute_forces(rbsog_handle *h, uint64_t step, const double *x_dev, double *f_dev,
                         double *f_near_dev, double *energy_dev);

/*
 * nsteps velocity-Verlet steps (Algorithm 2 time loop), in place:
 *   v += (dt/2) f / m;  x += dt v;  wrap into [0, L);  f = F(x, step0 + n + 1);
 *   v += (dt/2) f / m.
 * f_dev must hold F(x, step0) on entry (e.g. from rbsog_compute_forces).
 * energy_hist_dev (nullable, device) receives [nsteps][RBSOG_ENERGY_COLS]
 * energy rows of the new state, as in rbsog_compute_forces with
 * KE = sum m v^2 / 2 in slot 5.
 * A particle moving a box length or more in one step, or a non-finite force,
 * raises a device flag reported by rbsog_check.
 * Errors: RBSOG_EINVAL, RBSOG_EHIP.
 */
int rbsog_step(rbsog_handle *h, double *x_dev, double *v_dev, double *f_dev, uint64_t step0, int nsteps,
               double dt, double *energy_hist_dev);

/*
 * Instantaneous temperature in the sampling measure (Section 4.3: in NVT runs
 * the k_B T of the adaptive density, eq. 3.22, is the instantaneous one,
 * computed on the fly, while the other terms stay precomputed).  Re-derives
 * the shell CDF and the weights coef = S / (P V F(k)) of eq. 3.124 with kT in
 * place of the configured k_B T, on the host in the order rbsog_create uses,
 * and uploads them on the handle's stream: evaluations and steps enqueued
 * after this call draw from the new measure (modes drawn ahead are discarded),
 * those enqueued before it from the old one.  kT is typically 2 KE / (3N - 3)
 * from the last energy row.  The densities FLAT and K2 do not depend on kT
 * (their tables come out unchanged); with full_k only the stored kT changes.
 * Host work ~ one pass over the shells (<= 1e4); no stream synchronisation
 * except that a call waits for the previous call's upload to leave its pinned
 * staging buffer.  A higher kT re-runs the default skin's thermal check at the
 * next rbsog_step.  Errors: RBSOG_EINVAL (kT not positive and finite),
 * RBSOG_EHIP.
 */
int rbsog_set_kT(rbsog_handle *h, double kT);

/*
 * Thermostat of rbsog_step (Algorithm 2 leaves the integration scheme and
 * thermostat open; Section 5.1 runs NVT dynamics): a Langevin bath of
 * friction `friction` (per unit time) at temperature kT, as the BAOAB
 * splitting of the velocity-Verlet step -- the drift of each step becomes
 *   x += (dt/2) v;  v = c v + sqrt((1 - c^2) kT / m) z;  x += (dt/2) v,
 *   c = exp(-friction dt),
 * with z three standard normals per particle and step: Philox4x64-10(counter =
 * (caller index, force index the drift leads to, 1, 0), key = (seed,
 * replica)) as four uniforms ((w >> 11) + 1) 2^-53, through the Box-Muller
 * transform sqrt(-2 ln u0) (cos, sin)(2 pi u1), sqrt(-2 ln u2) cos(2 pi u3).
 * Reproducible and independent of the cell order.  friction = 0 (the
 * default) is plain velocity-Verlet (NVE).  The sampling measure keeps its
 * own temperature (rbsog_set_kT).  Single systems only (the served ensemble
 * runs NVE).  Errors: RBSOG_EINVAL (negative or non-finite friction, or kT not
 * positive and finite with friction > 0).
 */
int rbsog_set_thermostat(rbsog_handle *h, double friction, double kT);

#define RBSOG_BATH_NONE 0
#define RBSOG_BATH_LANGEVIN 1
#define RBSOG_BATH_NOSE_HOOVER 2
#define RBSOG_BATH_BERENDSEN 3

/*
 * Bath of rbsog_step, one at a time (replaces the previous one):
 *   RBSOG_BATH_NONE: plain velocity-Verlet (rate, kT ignored);
 *   RBSOG_BATH_LANGEVIN: as rbsog_set_thermostat(h, rate, kT);
 *   RBSOG_BATH_NOSE_HOOVER: the NVT dynamics Section 5.1 equilibrates with,
 *     one thermostat variable xi of mass Q = g kT tau^2 (g = 3N, tau = 1/rate);
 *   RBSOG_BATH_BERENDSEN: weak coupling, the kinetic energy relaxing to
 *     g kT/2 at rate 1/tau.
 * The global baths act as a half-step operator before and after each
 * velocity-Verlet step (with K the kinetic energy):
 *   Nose-Hoover: xi += (dt/4)(2K - g kT)/Q; v *= e^{-xi dt/2};
 *     eta += (dt/2) xi; xi += (dt/4)(2K - g kT)/Q (K after the scaling);
 *     K + U + Q xi^2/2 + g kT eta is conserved;
 *   Berendsen: v *= lambda, lambda^2 = 1 + (dt/(2 tau))(g kT/(2K) - 1).
 * The kinetic energy needs the whole system, so under a global bath each
 * step's next half-kick and drift run as a kernel of their own rather than in
 * the far kernel (one more launch and a single-workgroup reduction per step).
 * The energy rows report K after the step's closing half-step.  xi and eta
 * restart at 0 on every call that selects a global bath; they carry over
 * between rbsog_step calls.  Errors: RBSOG_EINVAL (unknown kind; rate or kT
 * not positive and finite for a bath other than NONE), RBSOG_EHIP.
 */
int rbsog_set_bath(rbsog_handle *h, int kind, double rate, double kT);

/*
 * The Nose-Hoover bath's state (the NVT runs of Section 5.1): its friction
 * xi and the integral eta of xi over time (which enters the conserved
 * extended energy K + U + Q xi^2/2 + g k_B T eta) into out[2] (host memory,
 * the caller's; meaningful for the Nose-Hoover bath only).  Synchronises the
 * stream.  Errors: RBSOG_EINVAL, RBSOG_EHIP.
 */
int rbsog_bath_state(rbsog_handle *h, double *out);

/*
 * Synchronises the stream and reports the device flag: RBSOG_OK, or
 * RBSOG_ENONFINITE if any evaluation since the last check produced a
 * non-finite force or an over-long step (the flag is then cleared).
 */
int rbsog_check(rbsog_handle *h);

/*
 * Per-kernel timing with HIP events recorded on the handle's stream around each
 * kernel launch (off by default; costs a few microseconds per launch when on).
 * Kernel classes, in slot order: 0 cell list (ids, scan, scatter, stable
 * rank + gather), 1 half-kick + drift, 2 mode sampling, 3 structure-factor
 * partials (a launch of their own: rbsog_compute_rho), 4 structure-factor
 * reduction, 5 near-field pair evaluation (in a force evaluation or step this
 * launch also computes the structure-factor partials, in its first
 * workgroups), 6 far field + force assembly + half-kick, 7 energy sums,
 * 8 near-field neighbour lists.
 */
#define RBSOG_NUM_KERNEL_CLASSES 9
typedef struct rbsog_timing {
    double ms[RBSOG_NUM_KERNEL_CLASSES];       /* summed event-to-event milliseconds */
    int64_t launches[RBSOG_NUM_KERNEL_CLASSES];
} rbsog_timing;

/* Turns timing on (enable != 0) or off and clears the accumulators.
 * Errors: RBSOG_EINVAL, RBSOG_EHIP. */
int rbsog_timing_enable(rbsog_handle *h, int enable);

/* Synchronises the stream, writes the accumulated times since the last
 * enable/read into *out and clears them.  Errors: RBSOG_EINVAL, RBSOG_EHIP. */
int rbsog_timing_read(rbsog_handle *h, rbsog_timing *out);

/* Releases the host-side handle (the caller still owns the workspace). */
void rbsog_destroy(rbsog_handle *h);

/* ------------------------------------------------------------------------
 * Served ensemble (Algorithm 2 for many independent systems at once)
 * ------------------------------------------------------------------------
 * Replicas -- independent systems of their own size, screening, temperature,
 * precision and seed, each running Algorithm 2 for a given number of steps --
 * are admitted into a device pool the ensemble owns, advanced together one
 * step per rbsog_ens_step (every step kernel is launched once for all active
 * replicas, over a (replica, workgroup) work list), and retired when done.
 * A replica's step n (n = 1 .. nsteps) is exactly the step of one system
 * (rbsog_step with step0 = 0): force-evaluation index 0 for the initial force,
 * computed at admission, and n for the force after the n-th drift, with the
 * replica's own seed and replica id keying the modes.  Not thread-safe: one
 * host thread drives an ensemble.  All device work is on the given stream. */
typedef struct rbsog_ens rbsog_ens;

/* Allocates the pool (hbm_budget bytes, rounded down to 256) and room for
 * max_slots resident replicas; the ensemble's own tables, work lists and the
 * shared Fourier lattice are allocated beside it.  Errors: RBSOG_EINVAL,
 * RBSOG_EHIP (the pool could not be allocated), RBSOG_ENOMEM. */
int rbsog_ens_create(size_t hbm_budget, int max_slots, void *hip_stream, rbsog_ens **out);

/* Pool bytes one replica with these parameters and step count occupies (its
 * workspace without the Fourier lattice, which the ensemble keeps once for
 * all replicas outside the pool, plus x, v, f, q, m and the energy history).
 * Errors: RBSOG_EINVAL. */
int rbsog_ens_bytes(const rbsog_params *p, const rbsog_sog *sog, int nsteps, size_t *bytes);

/* Admits one replica: copies x, v (SoA [3][N]), q, m ([N]) from host memory
 * into the pool, computes its initial force and queues it for nsteps steps of
 * length dt.  *slot_out receives its slot.  Synchronises the stream.
 * Errors: RBSOG_EAGAIN (no free slot, or no contiguous pool range for its
 * workspace + state + energy history: retry after a retirement),
 * RBSOG_EINVAL, RBSOG_ENOROOT, RBSOG_EHIP. */
int rbsog_ens_admit(rbsog_ens *e, const rbsog_params *p, const rbsog_sog *sog, const double *x_host,
                    const double *v_host, const double *q_host, const double *m_host, int nsteps, double dt,
                    int *slot_out);

/* Enqueues one step of every active replica (nothing when none is active);
 * asynchronous.  Errors: RBSOG_EINVAL, RBSOG_EHIP. */
int rbsog_ens_step(rbsog_ens *e);

/* Writes into done_slots (room for max_slots) the slots whose last step has
 * completed on the device and were not reported before; *n_done their count.
 * Does not wait.  Errors: RBSOG_EINVAL, RBSOG_EHIP. */
int rbsog_ens_poll(rbsog_ens *e, int *done_slots, int *n_done);

/* Copies a finished replica out (any of x_host, v_host [3][N] and
 * energy_hist_host [nsteps][RBSOG_ENERGY_COLS], rows as rbsog_compute_forces' energy_out of
 * steps 1..nsteps, may be null) and frees its slot and pool range.
 * Synchronises.  Errors: RBSOG_EINVAL (no such slot, or steps left),
 * RBSOG_ENONFINITE (the replica produced a non-finite force or an over-long
 * step; its slot is freed all the same), RBSOG_EHIP. */
int rbsog_ens_retire(rbsog_ens *e, int slot, double *x_host, double *v_host, double *energy_hist_host);

/* Resident replicas (active or finished, not yet retired), active replicas,
 * ensemble steps launched so far, free pool bytes (any may be null). */
int rbsog_ens_status(const rbsog_ens *e, int *resident, int *active, uint64_t *ens_steps, size_t *pool_free);

/* ------------------------------------------------------------------------
 * Observables (Section 5.1)
 * ------------------------------------------------------------------------ */

/* Scratch bytes rbsog_ssf needs for N particles and shells 1..m_s (host
 * only).  Errors: RBSOG_EINVAL. */
int rbsog_ssf_scratch_size(int64_t N, int m_s, size_t *bytes);

/*
 * Static structure factor by lattice shell (Section 5.1: S(k) = <rho(k) rho(-k)> / N
 * with rho the Fourier transform of the particle distribution), from the
 * structure-factor kernels of the far field over every lattice mode with
 * 1 <= |n|^2 <= m_s (k = 2 pi n / L, cubic box):
 *   s_dev[m] = (1/cnt_m) sum_{|n|^2 = m} |sum_j w_j exp(i k . r_j)|^2,
 * cnt_m the modes of shell m; s_dev[m] = 0 for m = 0 and for empty shells.
 * With unit weights w_dev, S(|k|) = s_dev / N; with the charges, the charge
 * structure factor.  x_dev [3][N] and w_dev [N] (device, caller order),
 * s_dev [m_s + 1] (device).  FP64 (sums in a fixed order, bitwise
 * reproducible).  scratch_dev: device memory of rbsog_ssf_scratch_size bytes,
 * 256-byte aligned, owned by the caller.  Work ~ N * (4/3) pi m_s^(3/2)
 * (particle, mode) terms.  Enqueued on hip_stream and synchronised before
 * returning (the host-side tables of the modes are released then).
 * Errors: RBSOG_EINVAL, RBSOG_EWORKSPACE, RBSOG_EHIP.
 */
int rbsog_ssf(int64_t N, double L, const double *x_dev, const double *w_dev, int m_s, void *scratch_dev,
              size_t scratch_bytes, void *hip_stream, double *s_dev);

/*
 * Pair-distance histogram behind the radial distribution function (Section
 * 5.1): for every ordered pair (i, j), i != j, with minimum-image distance
 * r < r_max, adds 1 to hist_dev[floor(r / dr)], dr = r_max / nbins (uint64,
 * device; the caller zeroes it, so that calls over many configurations
 * accumulate).  g(r) of bin b = hist[b] / (snapshots N (N / V) (4/3) pi
 * ((b + 1)^3 - b^3) dr^3).  x_dev [3][N] in [0, L) (device, caller order).
 * 0 < r_max <= r_c of the system, 1 <= nbins <= 4096.  Uses the system's fine
 * cell grid (its workspace rows are reordered; the next force evaluation
 * rebuilds its lists).  Integer counts, independent of the order of the
 * additions; a pair within rounding of a bin edge may fall on either side.
 * Asynchronous on the handle's stream.  Errors: RBSOG_EINVAL, RBSOG_EHIP.
 */
int rbsog_rdf(rbsog_handle *h, const double *x_dev, double r_max, int nbins, unsigned long long *hist_dev);

/*
 * Unwrapped displacements (for the mean squared displacement of Section 5.1):
 * disp_dev += d - L rint(d / L), d = x_dev - x_last_dev, then x_last_dev =
 * x_dev (all [3][N], device, caller order).  rbsog_step returns positions
 * wrapped into the box; calling this after each call (or often enough that no
 * particle moves L/2 or more in between) accumulates each particle's true
 * displacement.  Asynchronous on hip_stream.  Errors: RBSOG_EINVAL.
 */
int rbsog_track(int64_t N, double L, const double *x_dev, double *x_last_dev, double *disp_dev, void *hip_stream);

/*
 * rbsog_track in a cuboid box of edges (Lx, Ly, Lz) (Section 2's box
 * L = (L_x, L_y, L_z)): component a of d folds by its own edge, d - L_a
 * rint(d / L_a); arrays as rbsog_track ([3][N], device, caller order, owned
 * by the caller; x_last_dev and disp_dev updated in place).  Asynchronous on
 * hip_stream.  Errors: RBSOG_EINVAL (N outside [1, 2^27 - 1], an edge not
 * positive and finite, a null array).
 */
int rbsog_track_box(int64_t N, double Lx, double Ly, double Lz, const double *x_dev, double *x_last_dev,
                    double *disp_dev, void *hip_stream);

/* Scratch bytes of rbsog_msd_vacf (host only).  Errors: RBSOG_EINVAL. */
int rbsog_msd_scratch_size(size_t *bytes);

/*
 * Mean squared displacement and velocity autocorrelation at one time lag
 * (Section 5.1): out_dev[0] = (1/N) sum_i |disp_i|^2, out_dev[1] = (1/N)
 * sum_i v0_i . v_i (disp, v0, v [3][N], device; out [2], device), FP64 sums in
 * a fixed order (bitwise reproducible).  scratch_dev: rbsog_msd_scratch_size
 * bytes of device memory.  Asynchronous on hip_stream.
 * Errors: RBSOG_EINVAL, RBSOG_EWORKSPACE.
 */
int rbsog_msd_vacf(int64_t N, const double *disp_dev, const double *v0_dev, const double *v_dev, void *scratch_dev,
                   size_t scratch_bytes, void *hip_stream, double *out_dev);

/* Milliseconds from rbsog_ens_create to the device completion of ensemble
 * step ens_step (1-based, one of the last 8192 launched); waits for it.
 * Errors: RBSOG_EINVAL, RBSOG_EHIP. */
int rbsog_ens_step_time(rbsog_ens *e, uint64_t ens_step, double *ms);

/* Waits for the stream and frees the pool and every resident replica. */
void rbsog_ens_destroy(rbsog_ens *e);

/* ------------------------------------------------------------------------
 * Without allocation
 * ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * structure factors rho(k_l) = sum_j q_j exp(i k_l . r_j), k_l = 2 pi n_l / L,
 * of P given lattice modes n_dev[P][3] (int32, device), over N particles at
 * x_dev (SoA [3][N], caller order, device) with charges q_dev[N] (device),
 * written to rho_dev[P][2] = (re, im) (device) -- the sums rbsog_compute_rho
 * forms for the modes it draws, by the same kernels and group size, so the two
 * agree for the same modes.  No handle and no workspace: the modes as the
 * kernels read them, the rotation table, the partial sums and the reduction's
 * outputs live in one static 64 MiB device array that each GPU the library
 * runs on holds until the process ends; N and P whose partial sums would not
 * fit (about ceil(N / 256) * P * 16 bytes for large N) are refused with
 * RBSOG_EINVAL.  Calls no hipMalloc or hipFree.  The first call on a device
 * sets up (resolves the array's address on that device and copies the 2 KB
 * rotation table into it, synchronously) and must not be captured; later calls
 * only enqueue kernels on hip_stream.  Every call on one GPU shares its array
 * and overwrites what the last call left: calls that overlap on one GPU (other
 * streams, other host threads) race.  precision: RBSOG_FP64 or RBSOG_MIXED.
 * Errors: RBSOG_EINVAL, RBSOG_EHIP. */
int rbsog_rho_noalloc(int64_t N, double L, const double *x_dev, const double *q_dev, int P, const int32_t *n_dev,
                      int precision, void *hip_stream, double *rho_dev);

/* Thread-local message describing the last failing call. */
const char *rbsog_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RBSOG_H */

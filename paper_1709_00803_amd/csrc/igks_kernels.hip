// igks_kernels.hip - HIP kernels of the implicit gas-kinetic scheme for
// gfx950 (MI355X).
//
// One iteration = prep (per cell) -> flux (per face; each wave first takes
// the Eq.23 time step of its instance from the prep minima) -> gather (per
// cell) -> norm partial sums -> reduce (per instance: norms, Eq.25 CFL) ->
// forward sweep (one launch per wavefront) -> backward sweep with the state
// update -> commit (per instance).  No kernel waits on another inside a
// launch: ordering comes from launch boundaries only (device-scope fences
// inside a kernel would write back the XCD's whole L2).
//
// Data are structure-of-arrays in the library's internal cell order
// (wavefront, then instance, then upload index) and face order (interior
// faces, then boundary faces, each by their owner cell's position in the
// spatial-tile order of the cell kernels).  Face results go to per-face arrays and every cell sums its faces
// in a fixed order, so results are deterministic without floating-point
// atomics; the only atomics are integer min/max on the bit patterns of
// non-negative doubles.  Several independent instances (meshes and flow
// conditions) share every launch; each cell and face carries its instance.
#include "igks_dev.h"

#include <math.h>

namespace igks {

// ---------------------------------------------------------------- helpers

// 1/b for a positive finite b: the hardware reciprocal estimate refined by
// two Newton steps (each squares the relative error), to within about an
// ulp.  The flux kernels are bound by their FP64 instruction stream, and an
// IEEE FP64 divide is a sequence of about eleven instructions, this one of
// five.
__device__ __forceinline__ double frcp(double b)
{
    double x = __builtin_amdgcn_rcp(b);
    double e = fma(-b, x, 1.0);
    x = fma(e, x, x);
    e = fma(-b, x, 1.0);
    return fma(e, x, x);
}
// a/b (b positive, finite) from frcp with one residual correction
__device__ __forceinline__ double fdiv(double a, double b)
{
    const double x = frcp(b), q = a * x;
    return fma(fma(-b, q, a), x, q);
}
// 1/sqrt(a) for a positive finite a: the hardware estimate refined by two
// Newton steps of y <- y + y (1 - a y^2) / 2
__device__ __forceinline__ double frsq(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    double e = fma(-a * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-a * y, y, 1.0);
    return fma(0.5 * y, e, y);
}
// erfc(x).  For |x| <= 1 (every face of a subsonic flow: x = sqrt(lambda) U
// is about 0.84 times the local normal Mach number) from the Maclaurin series
// of erf (Abramowitz & Stegun 7.1.5), erf(x) = 2/sqrt(pi) sum_n (-1)^n
// x^(2n+1) / (n! (2n+1)), 18 terms summed by Horner's rule in x^2 (the first
// term left out is below 5e-18 of erf(1)); erfc = 1 - erf lies in [0.15, 1.85]
// there, so nothing cancels.  Beyond, the library erfc.  The series costs a
// seventh of the library's instruction sequence.
struct ErfSeries {
    double c[18];
};
constexpr ErfSeries erf_series()
{
    ErfSeries s{};
    double f = 1.0;   // n!, exact up to 18!
    for (int n = 0; n < 18; n++) {
        if (n > 0) f *= n;
        s.c[n] = (n % 2 ? -M_2_SQRTPI : M_2_SQRTPI) / (f * (2 * n + 1));
    }
    return s;
}
__device__ __forceinline__ double erfc_s(double x)
{
    if (fabs(x) <= 1.0) {
        constexpr ErfSeries S = erf_series();
        const double z = x * x;
        double p = S.c[17];
#pragma unroll
        for (int n = 16; n >= 0; n--) p = fma(p, z, S.c[n]);
        return 1.0 - x * p;
    }
    return erfc(x);
}

// 1/(2 lambda) of a conservative state (rho, rho U, rho V, rho E) from its
// 1/rho: lambda = (K+2) rho / (4 (rho E - rho |U|^2 / 2)) (Sec. 2.1, Eq.2),
// so 1/(2 lambda) = 2 (rho E - rho |U|^2 / 2) / ((K+2) rho), no divide.
__device__ __forceinline__ double half_inv_lam(const double *w, double ir)
{
    return (2.0 / (KDOF + 2.0)) * (w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) * ir) * ir;
}

// Sutherland's law relative to the 288.15 K free stream, T/T_inf = lam_inf/lam.
__device__ __forceinline__ double mu_lam(int law, const InstParam &ip, double lam)
{
    if (law) return ip.mu_inf;
    const double S = 110.4 / 288.15;
    double th = ip.lam_inf / lam;
    return ip.mu_inf * th * sqrt(th) * (1.0 + S) / (th + S);
}

__device__ __forceinline__ double lam_of(const double *w)
{
    double r = w[0], U = w[1] / r, V = w[2] / r;
    return (KDOF + 2.0) * r / (4.0 * (w[3] - 0.5 * r * (U * U + V * V)));
}

__device__ __forceinline__ double sa_fv1(double chi)
{
    double c3 = chi * chi * chi;
    return c3 / (c3 + 7.1 * 7.1 * 7.1);
}
// The same two laws for the flux kernels: the viscosity from hl = 1/(2
// lambda) (T/T_inf = 2 lam_inf hl), and f_v1, with frcp / frsq in place of
// the IEEE divides and square roots.
__device__ __forceinline__ double mu_hl(int law, const InstParam &ip, double hl)
{
    if (law) return ip.mu_inf;
    const double S = 110.4 / 288.15;
    const double th = 2.0 * ip.lam_inf * hl;
    return ip.mu_inf * (1.0 + S) * (th * th * frsq(th)) * frcp(th + S);
}
__device__ __forceinline__ double sa_fv1_f(double chi)
{
    double c3 = chi * chi * chi;
    return c3 * frcp(c3 + 7.1 * 7.1 * 7.1);
}

// SA constants (standard model without the f_t2 term)
#define SA_CB1 0.1355
#define SA_CB2 0.622
#define SA_SIGMA (2.0 / 3.0)
#define SA_KAPPA 0.41
#define SA_CW2 0.3
#define SA_CW3 2.0

// Eq.28a source and the non-negative part of -dSr/dnu~ (implicit diagonal).
__device__ __forceinline__ void sa_source(double nut, double nu, double d, double om, double &Sr, double &jd)
{
    const double cw1 = SA_CB1 / (SA_KAPPA * SA_KAPPA) + (1.0 + SA_CB2) / SA_SIGMA;
    double k2d2 = SA_KAPPA * SA_KAPPA * d * d;
    double chi = nut / nu;
    double fv2 = 1.0 - chi / (1.0 + chi * sa_fv1(chi));
    double Sb = nut * fv2 / k2d2;
    double St = (Sb >= -0.7 * om) ? om + Sb : om + om * (0.49 * om + 0.9 * Sb) / ((0.9 - 1.4) * om - Sb);
    double r = (St > 0.0) ? nut / (St * k2d2) : 10.0;
    r = fmin(r, 10.0);
    double r2 = r * r, r6 = r2 * r2 * r2;
    double g = r + SA_CW2 * (r6 - r);
    double g2 = g * g, g6 = g2 * g2 * g2;
    const double c6 = 64.0;   // c_w3^6
    double fw = g * pow((1.0 + c6) / (g6 + c6), 1.0 / 6.0);
    Sr = SA_CB1 * St * nut - cw1 * fw * (nut / d) * (nut / d);
    jd = fmax(2.0 * cw1 * fw * nut / (d * d) - SA_CB1 * St, 0.0);
}

// Ghost cell-centre state across a boundary face with outward unit normal n
// (Sec. 2.5).
// speed of a moving wall along the face tangent t = (-n_y, n_x): the
// free-stream velocity's tangential component
__device__ __forceinline__ double wall_speed(const InstParam &ip, double nx, double ny)
{
    return (ip.Winf[1] * -ny + ip.Winf[2] * nx) / ip.Winf[0];
}

// cell-centre ghost of an isothermal no-slip wall: the interior pressure,
// RT mirrored about the wall's (2 RT_w - RT, at least RT_w / 2), the
// no-slip ghost velocity (ux, uy), nu-tilde negated
__device__ __forceinline__ void iso_ghost(const InstParam &ip, const double *w, double ux, double uy, double *g)
{
    const double p = (GAMMA - 1.0) * (w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0]);
    const double tg = fmax(2.0 * ip.tw - p / w[0], 0.5 * ip.tw);
    const double rg = p / tg;
    g[0] = rg;
    g[1] = rg * ux;
    g[2] = rg * uy;
    g[3] = p * (1.0 / (GAMMA - 1.0)) + 0.5 * rg * (ux * ux + uy * uy);
    g[4] = -w[4];
}

__device__ __forceinline__ void ghost(const InstParam &ip, int bc, const double *w, double nx, double ny, double *g)
{
    if (bc == BC_FREESTREAM) {
#pragma unroll
        for (int k = 0; k < 5; k++) g[k] = ip.Winf[k];
        return;
    }
    double r = w[0], mx = w[1], my = w[2];
    if (bc == BC_SYMMETRY) {
        double mn = mx * nx + my * ny;
        g[0] = r; g[1] = mx - 2.0 * mn * nx; g[2] = my - 2.0 * mn * ny; g[3] = w[3]; g[4] = w[4];
        return;
    }
    if (bc == BC_WALL) {
        if (ip.tw > 0.0) { iso_ghost(ip, w, -mx / r, -my / r, g); return; }
        g[0] = r; g[1] = -mx; g[2] = -my; g[3] = w[3]; g[4] = -w[4];
        return;
    }
    if (bc == BC_MOVING_WALL) {
        // no-slip wall moving with the tangential part V_w of the free-stream
        // velocity: interior density and temperature, velocity 2 V_w - V
        double vt = wall_speed(ip, nx, ny), vwx = -vt * ny, vwy = vt * nx;
        if (ip.tw > 0.0) { iso_ghost(ip, w, 2.0 * vwx - mx / r, 2.0 * vwy - my / r, g); return; }
        g[0] = r;
        g[1] = 2.0 * vwx * r - mx;
        g[2] = 2.0 * vwy * r - my;
        g[3] = w[3] + 2.0 * r * (vwx * vwx + vwy * vwy) - 2.0 * (vwx * mx + vwy * my);
        g[4] = -w[4];
        return;
    }
    // Riemann-invariant outflow: U_b from R+ (inside) and R- (free stream),
    // rho and lam from inside, tangential velocity from inside.
    double U = mx / r, V = my / r, lam = lam_of(w);
    double ci = sqrt(GAMMA / (2.0 * lam));
    double co = sqrt(GAMMA / (2.0 * ip.lam_inf));
    double Ui = U * nx + V * ny;
    double Uo = ip.Winf[1] * nx + ip.Winf[2] * ny;
    double Ub = 0.5 * ((Ui + 2.0 * ci / (GAMMA - 1.0)) + (Uo - 2.0 * co / (GAMMA - 1.0)));
    double Vt = -U * ny + V * nx;
    g[0] = r;
    g[1] = r * (Ub * nx - Vt * ny);
    g[2] = r * (Ub * ny + Vt * nx);
    g[3] = 0.5 * r * (Ub * Ub + Vt * Vt + (KDOF + 2.0) / (2.0 * lam));
    g[4] = w[4];
}

// ghost increments (Sec. 2.5)
template <typename V>
__device__ __forceinline__ void ghost_incr(int bc, const V *d, V nx, V ny, V vw, V *g)
{
    if (bc == BC_MOVING_WALL) {   // the linear map of the moving-wall ghost; vw = wall speed along t
        V vwx = -vw * ny, vwy = vw * nx;
        g[0] = d[0];
        g[1] = V(2) * vwx * d[0] - d[1];
        g[2] = V(2) * vwy * d[0] - d[2];
        g[3] = d[3] + V(2) * (vwx * vwx + vwy * vwy) * d[0] - V(2) * (vwx * d[1] + vwy * d[2]);
        g[4] = -d[4];
        return;
    }
    if (bc == BC_SYMMETRY) {
        V mn = d[1] * nx + d[2] * ny;
        g[0] = d[0]; g[1] = d[1] - V(2) * mn * nx; g[2] = d[2] - V(2) * mn * ny; g[3] = d[3]; g[4] = d[4];
    } else if (bc == BC_WALL) {
        g[0] = d[0]; g[1] = -d[1]; g[2] = -d[2]; g[3] = d[3]; g[4] = -d[4];
    } else {
#pragma unroll
        for (int k = 0; k < 5; k++) g[k] = V(0);
    }
}

// Block index remapped so that each XCD works on one contiguous range of
// cells or faces (workgroups are dealt to the 8 XCDs in turn, and each XCD
// has its own L2): neighbour data of a range then stay in one L2.  A
// bijection of [0, gridDim.x) whatever the dealing order.
__device__ __forceinline__ int xcd_block()
{
    const int nxcd = 8;
    int nb = (int)gridDim.x, b = (int)blockIdx.x;
    int q = nb / nxcd, r = nb % nxcd, x = b % nxcd;
    return x * q + min(x, r) + b / nxcd;
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = warpSize / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = warpSize / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// slot s of quantity `kind` of instance `inst`
__device__ __forceinline__ unsigned long long *slot_at(unsigned long long *slot, int inst, int kind, int s)
{
    return slot + ((size_t)(inst * NSL + kind) * NSLOT + s) * SLOT_STRIDE;
}
// the lane's slot (lane mod NSLOT) of quantity `kind` of instance `inst`, as a double
__device__ __forceinline__ double slot_lane(const unsigned long long *slot, int inst, int kind)
{
    const int lane = (int)(threadIdx.x & (warpSize - 1)) & (NSLOT - 1);
    return __longlong_as_double((long long)slot[((size_t)(inst * NSL + kind) * NSLOT + lane) * SLOT_STRIDE]);
}

// Atomic min / max of a non-negative double into one of the NSLOT slots of
// the lane's instance.  Lanes with inst < 0 take no part.  When the whole
// wave belongs to one instance it combines first and issues one atomic.
template <bool MIN>
__device__ __forceinline__ void slot_update(unsigned long long *slot, int kind, int inst, double v)
{
    unsigned long long act = __ballot(inst >= 0);
    if (act == 0ull) return;
    int src = __ffsll((long long)act) - 1;
    int i0 = __shfl(inst, src);
    int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) / warpSize);
    int s = wave & (NSLOT - 1);
    if (__all(inst < 0 || inst == i0)) {
        double x = (inst >= 0) ? v : (MIN ? INFINITY : 0.0);
        x = MIN ? wave_min(x) : wave_max(x);
        if ((int)(threadIdx.x & (warpSize - 1)) == src) {
            unsigned long long *p = slot_at(slot, i0, kind, s);
            if (MIN) atomicMin(p, (unsigned long long)__double_as_longlong(x));
            else atomicMax(p, (unsigned long long)__double_as_longlong(x));
        }
    } else if (inst >= 0) {
        unsigned long long *p = slot_at(slot, inst, kind, s);
        if (MIN) atomicMin(p, (unsigned long long)__double_as_longlong(v));
        else atomicMax(p, (unsigned long long)__double_as_longlong(v));
    }
}

__device__ __forceinline__ double slots_min_serial(const unsigned long long *slot, int inst, int kind)
{
    double v = INFINITY;
    for (int i = 0; i < NSLOT; i++)
        v = fmin(v, __longlong_as_double((long long)slot[((size_t)(inst * NSL + kind) * NSLOT + i) * SLOT_STRIDE]));
    return v;
}

// One block of four cell-face entries (block b: the cell's own block b = c,
// or a polygon's overflow block): face, neighbour (-1: ghost) and flags,
// one 16-byte load each.
struct Entries {
    int face[MAXV], nbr[MAXV], flag[MAXV];
};
template <typename T>
__device__ __forceinline__ Entries entries(const Params<T> &P, int b)
{
    const int4 f = reinterpret_cast<const int4 *>(P.cf_face)[b];
    const int4 n = reinterpret_cast<const int4 *>(P.cf_nbr)[b];
    const int4 g = reinterpret_cast<const int4 *>(P.cf_flag)[b];
    return Entries{{f.x, f.y, f.z, f.w}, {n.x, n.y, n.z, n.w}, {g.x, g.y, g.z, g.w}};
}
// the block after E, or -1 (triangles and quadrilaterals have one block)
template <typename T>
__device__ __forceinline__ int next_block(const Params<T> &P, const Entries &E)
{
    const int o = E.flag[MAXV - 1] >> CF_NEXT_SHIFT;
    return o ? P.nc + o - 1 : -1;
}

// instance of a cell / face (a one-instance context needs no lookup)
template <typename T>
__device__ __forceinline__ int cell_inst(const Params<T> &P, int c)
{
    return P.ninst == 1 ? 0 : P.cinst[c];
}
// The instance a cell (or face) works for, -1 if it is frozen.  ONE: a
// context of one instance.  Its index is the constant 0, so the instance's
// scalars come through scalar loads, and the frozen flag is not consulted:
// a frozen instance's current state buffer is never written again (the
// update goes to the other buffer and the commit does not flip it), so
// recomputing its residual and increment changes nothing, while the check
// would put a dependent load in front of every other load of the kernel.
template <bool ONE, typename T>
__device__ __forceinline__ int live_inst(const Params<T> &P, const int *idx, int i)
{
    if (ONE) return 0;
    const int inst = P.ninst == 1 ? 0 : idx[i];
    return P.is[inst].halt ? -1 : inst;
}
template <typename T>
__device__ __forceinline__ int face_inst(const Params<T> &P, int f)
{
    return P.ninst == 1 ? 0 : P.finst[f];
}

template <typename T>
__device__ __forceinline__ const double *cur_state(const Params<T> &P, int inst)
{
    return (P.is[inst].ncommit & 1) ? P.Wb : P.Wa;
}

// ------------------------------------------------------- kinetic building blocks

// <u^k>, k = 0..7, of the normalised Maxwellian exp(-lam (u-U)^2) on the
// whole line (S = 0), on u > 0 (S = +1) or on u < 0 (S = -1); hl = 1/(2 lam)
// (the moment helpers take it precomputed: one divide per Maxwellian).
template <int S>
__device__ __forceinline__ void mom_u(double U, double lam, double hl, double *m)
{
    if (S == 0) {
        m[0] = 1.0; m[1] = U;
    } else {
        double x = sqrt(lam) * U;
        double e = exp(-x * x) * (0.5 / sqrt(M_PI * lam));
        if (S > 0) { m[0] = 0.5 * erfc(-x); m[1] = U * m[0] + e; }
        else { m[0] = 0.5 * erfc(x); m[1] = U * m[0] - e; }
    }
#pragma unroll
    for (int k = 0; k < 6; k++) m[k + 2] = U * m[k + 1] + (k + 1) * hl * m[k];
}
// The same half-space moments with the half chosen at run time: sgn = +1
// for u > 0, -1 for u < 0 (the two lanes of a face take opposite halves).
// SERIES: erfc from erfc_s (the sides' Maxwellians); otherwise the library
// erfc (the equilibrium state's half spaces: the series there too raised the
// one-lane flux kernel from 242 to 283 registers, one wave per SIMD instead
// of two).
template <bool SERIES>
__device__ __forceinline__ void mom_u_half(double U, double lam, double hl, double sgn, double *m)
{
    // one refined 1/sqrt(lam) gives both sqrt(lam) and 1/sqrt(pi lam)
    const double s = frsq(lam);
    double x = lam * s * U;
    double e = exp(-x * x) * (0.5 / sqrt(M_PI)) * s;
    // the sign is applied by selection, not by a product, so that m[1] is
    // formed the same way whether sgn is known at compile time or not
    double es = sgn > 0.0 ? e : -e, xs = sgn > 0.0 ? -x : x;
    m[0] = 0.5 * (SERIES ? erfc_s(xs) : erfc(xs));
    m[1] = U * m[0] + es;
#pragma unroll
    for (int k = 0; k < 6; k++) m[k + 2] = U * m[k + 1] + (k + 1) * hl * m[k];
}
// <xi^0>, <xi^2>, <xi^4> over K internal dimensions
__device__ __forceinline__ void mom_xi(double hl, double *x)
{
    x[0] = 1.0;
    x[1] = KDOF * hl;
    x[2] = x[1] * (KDOF + 2.0) * hl;
}

// Moments out = < u^A v^B (c0 + c1 u + c2 v + c3 (u^2+v^2+xi^2)/2) psi > with
// psi = (1, u, v, (u^2+v^2+xi^2)/2) of a Maxwellian, from its u, v and xi
// moment arrays mu, mv, mx (exponents compile-time, so the arrays stay in
// registers).  The velocity-space sums are regrouped by powers of u: with
// G0 = c0 + c2 v + c3 H, G1 = c1, G2 = c3 / 2 and H = (v^2 + xi^2) / 2 the
// weight is sum_k u^k G_k and psi_3 = u^2 / 2 + H, so
//   out0 = sum_k <u^(A+k)> <v^B G_k>,      out1 = sum_k <u^(A+1+k)> <v^B G_k>,
//   out2 = sum_k <u^(A+k)> <v^(B+1) G_k>,
//   out3 = sum_k (<u^(A+2+k)> <v^B G_k> / 2 + <u^(A+k)> <v^B H G_k>).
// The nine v, xi factors depend on the Maxwellian's v and xi moments and on
// c only, so one set serves the u-moments of both half spaces and of the
// whole line, and every exponent A: vx_coef forms them once, vx_apply
// combines them with one set of u-moments (15 multiply-adds).
struct VX {
    double g[3], gp[3], h[3];   // <v^B G_k>, <v^(B+1) G_k>, <v^B H G_k>
};
template <int B>
__device__ __forceinline__ VX vx_coef(const double *mv, const double *mx, const double *c)
{
    // <v^B H>, <v^(B+1) H>, <v^B H^2>
    const double e0 = 0.5 * (mv[B + 2] + mv[B] * mx[1]);
    const double e1 = 0.5 * (mv[B + 3] + mv[B + 1] * mx[1]);
    const double e2 = 0.25 * (mv[B + 4] + 2.0 * mv[B + 2] * mx[1] + mv[B] * mx[2]);
    VX o;
    o.g[0] = c[0] * mv[B] + c[2] * mv[B + 1] + c[3] * e0;
    o.g[1] = c[1] * mv[B];
    o.g[2] = 0.5 * c[3] * mv[B];
    o.gp[0] = c[0] * mv[B + 1] + c[2] * mv[B + 2] + c[3] * e1;
    o.gp[1] = c[1] * mv[B + 1];
    o.gp[2] = 0.5 * c[3] * mv[B + 1];
    o.h[0] = c[0] * e0 + c[2] * e1 + c[3] * e2;
    o.h[1] = c[1] * e0;
    o.h[2] = 0.5 * c[3] * e0;
    return o;
}
template <int A>
__device__ __forceinline__ void vx_apply(const double *mu, const VX &o, double *out)
{
    out[0] = mu[A] * o.g[0] + mu[A + 1] * o.g[1] + mu[A + 2] * o.g[2];
    out[1] = mu[A + 1] * o.g[0] + mu[A + 2] * o.g[1] + mu[A + 3] * o.g[2];
    out[2] = mu[A] * o.gp[0] + mu[A + 1] * o.gp[1] + mu[A + 2] * o.gp[2];
    out[3] = 0.5 * (mu[A + 2] * o.g[0] + mu[A + 3] * o.g[1] + mu[A + 4] * o.g[2]) + mu[A] * o.h[0] +
             mu[A + 1] * o.h[1] + mu[A + 2] * o.h[2];
}

// <u^A psi>
template <int A>
__device__ __forceinline__ void pmom1(const double *mu, const double *mv, const double *mx, double *out)
{
    out[0] = mu[A];
    out[1] = mu[A + 1];
    out[2] = mu[A] * mv[1];
    out[3] = 0.5 * (mu[A + 2] + mu[A] * mv[2] + mu[A] * mx[1]);
}

// Closed-form solution of M(g) a = b for the Maxwellian moment matrix
// M_ij = <psi_i psi_j> (the Sec. 2.1 moment relations after Eq.4, divided
// by rho), in the closed form of Xu's BGK scheme (Xu 2001, J. Comput. Phys.).
__device__ __forceinline__ void msolve(double U, double V, double lam, double hl, const double *b, double *a)
{
    double B = U * U + V * V + (KDOF + 2.0) * hl;
    double R2 = b[1] - U * b[0], R3 = b[2] - V * b[0], R4 = 2.0 * b[3] - B * b[0];
    a[3] = lam * lam * (4.0 / (KDOF + 2.0)) * (R4 - 2.0 * U * R2 - 2.0 * V * R3);
    a[2] = 2.0 * lam * R3 - V * a[3];
    a[1] = 2.0 * lam * R2 - U * a[3];
    a[0] = b[0] - U * a[1] - V * a[2] - 0.5 * a[3] * B;
}

// Value of the partner lane of a face's lane pair (lanes 2m and 2m + 1): a
// DPP quad permutation [1, 0, 3, 2] on each 32-bit half, which moves the
// value between neighbouring lanes inside the VALU instead of through the
// LDS crossbar.  Both lanes of a pair are active together.
__device__ __forceinline__ int pair_swap(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);
}
__device__ __forceinline__ double pair_other(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = pair_swap((int)(b & 0xffffffffll)), hi = pair_swap((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// a + b rounded once and never fused with the product that produced a or b:
// the sum of a face's two sides is then the same number on either lane of a
// pair and in the one-lane kernel (a fused multiply-add would round
// differently depending on which side's product it absorbed).
__device__ __forceinline__ double add_sides(double a, double b)
{
#pragma clang fp contract(off)
    return a + b;
}

// One side's part of the interface distribution that does not depend on the
// equilibrium state: slopes a_n, a_t (Eq.4 and the moment relations after it), A (Eq.11) and the
// half-space moments that multiply them, for the left state on u > 0
// (sgn = +1) or the right state on u < 0 (sgn = -1).  Writes (rho-weighted)
//   acc[0..3] = <psi>, acc[4..7] = <(u a_n + v a_t) psi>, acc[8..11] = <A psi>,
//   acc[12..15] = <u psi>, acc[16..19] = <u (u a_n + v a_t) psi>, acc[20..23] = <u A psi>.
__device__ __forceinline__ void side_terms(double sgn, const double *w, const double *gn, const double *gt,
                                           double *acc)
{
    // one reciprocal per denominator: an FP64 divide is a long sequence,
    // and the flux kernels are bound by their FP64 instruction stream
    double r = w[0], ir = frcp(r), U = w[1] * ir, V = w[2] * ir, hl = half_inv_lam(w, ir), lam = 0.5 * frcp(hl);
    double an[4], at[4], A[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; k++) b[k] = gn[k] * ir;
    msolve(U, V, lam, hl, b, an);
#pragma unroll
    for (int k = 0; k < 4; k++) b[k] = gt[k] * ir;
    msolve(U, V, lam, hl, b, at);
    double mv[8], mx[3], mu[8], mf[8];
    mom_u<0>(V, lam, hl, mv);
    mom_xi(hl, mx);
    mom_u<0>(U, lam, hl, mf);
    mom_u_half<true>(U, lam, hl, sgn, mu);
    double t[4], s[4], t4[4], t16[4];
    {
        // a_n: <u a_n psi> over the whole line (for A) and on the half
        // space, <u^2 a_n psi> on the half space
        const VX x = vx_coef<0>(mv, mx, an);
        vx_apply<1>(mf, x, b);
        vx_apply<1>(mu, x, t4);
        vx_apply<2>(mu, x, t16);
    }
    {
        // a_t: the same with v in place of u
        const VX x = vx_coef<1>(mv, mx, at);
        vx_apply<0>(mf, x, t);
#pragma unroll
        for (int k = 0; k < 4; k++) b[k] = -(b[k] + t[k]);
        vx_apply<0>(mu, x, t);
        vx_apply<1>(mu, x, s);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            acc[4 + k] = r * (t4[k] + t[k]);
            acc[16 + k] = r * (t16[k] + s[k]);
        }
    }
    msolve(U, V, lam, hl, b, A);
    {
        const VX x = vx_coef<0>(mv, mx, A);
        vx_apply<0>(mu, x, t);
        vx_apply<1>(mu, x, s);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            acc[8 + k] = r * t[k];
            acc[20 + k] = r * s[k];
        }
    }
    pmom1<0>(mu, mv, mx, t);
    pmom1<1>(mu, mv, mx, s);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        acc[k] = r * t[k];
        acc[12 + k] = r * s[k];
    }
}

// Equilibrium part of the interface (Eq.4-5, Eq.11-14), split so that the
// two half spaces can be evaluated on one lane or on the two lanes of a
// face.  gks_eq: g0 from the summed side moments, the Eq.34 collision time
// and the time integrals of the six Eq.13 factors over [0, dt].
struct GksEq {
    double r0, U0, V0, lam0, ir0, hl0;
    double T1, T2, T3, T4, T5, T6;
    double mv[8], mx[3];
};
template <typename T>
__device__ __forceinline__ void gks_eq(const Params<T> &P, const InstParam &ip, const double *w0, double dt,
                                       double nut_f, double jump, GksEq &q)
{
    q.r0 = w0[0];
    q.ir0 = frcp(q.r0);
    q.U0 = w0[1] * q.ir0; q.V0 = w0[2] * q.ir0; q.hl0 = half_inv_lam(w0, q.ir0); q.lam0 = 0.5 * frcp(q.hl0);
    double mul = mu_hl(P.mu_law, ip, q.hl0), mut = 0.0;
    if (ip.sa && nut_f > 0.0) mut = q.r0 * nut_f * sa_fv1_f(nut_f * q.r0 * frcp(mul));
    double tau = (mul + mut) * 2.0 * q.lam0 * q.ir0;
    if (P.tau_jump) tau += dt * jump;
    const double x = dt * frcp(tau);
    double eta = exp(-x), ome = -expm1(-x);
    q.T1 = dt - tau * ome;
    q.T2 = -tau * dt * (1.0 + eta) + 2.0 * tau * tau * ome;
    q.T3 = 0.5 * dt * dt - tau * dt + tau * tau * ome;
    q.T4 = tau * ome;
    q.T5 = tau * dt * eta - 2.0 * tau * tau * ome;
    q.T6 = -tau * tau * ome;
    mom_u<0>(q.V0, q.lam0, q.hl0, q.mv);
    mom_xi(q.hl0, q.mx);
}
// One half space of q2 = <psi (abar_n H u + abar_n' (1-H) u)> and of its flux
// moment f2 = <u psi (...)>: left (sgn = +1) with the slope (W0 - W_l)/d_l
// on u > 0, right (sgn = -1) with (W_r - W0)/d_r on u < 0.
__device__ __forceinline__ void gks_half(const GksEq &q, double sgn, const double *w0, const double *wc, double id,
                                         double *q2, double *f2)
{
    double b[4], a[4], mh[8];
    const double sd = q.ir0 * id;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        double dw = sgn > 0.0 ? w0[k] - wc[k] : wc[k] - w0[k];
        b[k] = dw * sd;
    }
    msolve(q.U0, q.V0, q.lam0, q.hl0, b, a);
    mom_u_half<false>(q.U0, q.lam0, q.hl0, sgn, mh);
    const VX x = vx_coef<0>(q.mv, q.mx, a);
    vx_apply<1>(mh, x, q2);
    vx_apply<2>(mh, x, f2);
}
// The rest, from the summed side moments acc, the summed half-space q2 and
// f2, and the sum of the two sides' tangential slopes: the abar_t term,
// Abar from Eq.12 and the flux of Eq.14 integrated over [0, dt].
__device__ __forceinline__ void gks_finish(const GksEq &q, const double *acc, double *q2, double *f2,
                                           const double *gt_sum, double dt, double *F)
{
    const double *q5 = acc + 4, *q6 = acc + 8, *f4 = acc + 12, *f5 = acc + 16, *f6 = acc + 20;
    double mf[8], a[4], b[4], t[4];
    mom_u<0>(q.U0, q.lam0, q.hl0, mf);
#pragma unroll
    for (int k = 0; k < 4; k++) b[k] = 0.5 * gt_sum[k] * q.ir0;
    msolve(q.U0, q.V0, q.lam0, q.hl0, b, a);
    {
        const VX x = vx_coef<1>(q.mv, q.mx, a);
        vx_apply<0>(mf, x, t);
#pragma unroll
        for (int k = 0; k < 4; k++) q2[k] = q.r0 * (q2[k] + t[k]);
        vx_apply<1>(mf, x, t);
#pragma unroll
        for (int k = 0; k < 4; k++) f2[k] += t[k];
    }
    // Eq.12 -> Abar
    const double iden = frcp(q.r0 * (0.5 * dt * dt - q.T3));
#pragma unroll
    for (int k = 0; k < 4; k++) b[k] = (q.T2 * q2[k] + q.T5 * q5[k] + q.T6 * q6[k]) * iden;
    msolve(q.U0, q.V0, q.lam0, q.hl0, b, a);
    // Eq.14
    double e1[4];
    pmom1<1>(mf, q.mv, q.mx, e1);
    vx_apply<1>(mf, vx_coef<0>(q.mv, q.mx, a), t);
#pragma unroll
    for (int k = 0; k < 4; k++)
        F[k] = q.T1 * q.r0 * e1[k] + q.T2 * q.r0 * f2[k] + q.T3 * q.r0 * t[k] + q.T4 * f4[k] + q.T5 * f5[k] +
               q.T6 * f6[k];
}

// Euler flux Jacobian-vector product J(W, n) d (the linearised flux of the
// implicit operator, Eq.18-20).  One reciprocal of rho: the sweeps run one
// wavefront after another, and a divide is a long dependent sequence.
template <typename V>
__device__ __forceinline__ void jac_vec(const V *W, V nx, V ny, const V *d, V *out)
{
    V r = W[0], ir = V(1) / r, U = W[1] * ir, Vv = W[2] * ir, E = W[3];
    V ke = V(0.5) * (U * U + Vv * Vv);
    V p = V(GAMMA - 1.0) * (E - r * ke);
    V q = U * nx + Vv * ny;
    V dmn = d[1] * nx + d[2] * ny;
    V dq = (dmn - q * d[0]) * ir;
    V dp = V(GAMMA - 1.0) * (d[3] - (U * d[1] + Vv * d[2]) + ke * d[0]);
    out[0] = dmn;
    out[1] = d[1] * q + W[1] * dq + dp * nx;
    out[2] = d[2] * q + W[2] * dq + dp * ny;
    out[3] = (d[3] + dp) * q + (E + p) * dq;
}

// ------------------------------------------------------------------ kernels

// mode bit 1: per-iteration slots; 2: bad/halt flags; 8: all scalars of the
// instance (fresh start).  inst < 0: every instance.
template <typename T>
__global__ void k_reset(Params<T> P, int mode, int inst)
{
    int lo = inst < 0 ? 0 : inst, hi = inst < 0 ? P.ninst : inst + 1;
    for (int i = lo + (int)threadIdx.x; i < hi; i += blockDim.x) {
        InstScalars *s = &P.is[i];
        if (mode & 8) {
            s->dt = s->cfl = s->res_inf_prev = s->res0 = 0.0;
            s->res_l2 = s->sa_l2 = s->res_inf = s->e40 = 0.0;
            s->ncommit = 0;
        }
        if (mode & (1 | 8))
            for (int k = 0; k < NSLOT; k++) {
                *slot_at(P.slot, i, SL_DTMIN, k) = 0x7ff0000000000000ull;   // +inf
                *slot_at(P.slot, i, SL_RESINF, k) = 0ull;
                *slot_at(P.slot, i, SL_E40, k) = 0ull;
            }
        if (mode & (2 | 8)) { s->bad = 0; s->halt = 0; }
    }
}

// Per cell: Eq.21 spectral radius and the Eq.23 time step, least-squares
// gradients (Eq.6-7, ghost cells included), the Eq.9-10 limiter,
// vorticity and the laminar viscosity.
template <typename T>
__device__ __forceinline__ double prep_cell(const Params<T> &P, int c, int inst)
{
    const int N = P.nc;
    const InstParam &ip = P.ip[inst];
    const double *W = cur_state(P, inst);
    double w[5];
#pragma unroll
    for (int k = 0; k < 5; k++) w[k] = W[k * N + c];
    double r = w[0], U = w[1] / r, V = w[2] / r;
    double lam = lam_of(w);
    double cs = sqrt(GAMMA / (2.0 * lam));
    P.nu[c] = mu_lam(P.mu_law, ip, lam) / r;
    double lc = 0.0, b1[4] = {0, 0, 0, 0}, b2[4] = {0, 0, 0, 0}, wmax[4], wmin[4];
#pragma unroll
    for (int k = 0; k < 4; k++) wmax[k] = wmin[k] = w[k];
    // the cell's block, then a polygon's overflow block (a rarely taken branch,
    // so triangles and quadrilaterals run straight-line code)
    auto block = [&](const Entries &E, int b) {
#pragma unroll
        for (int k = 0; k < MAXV; k++) {
            if (!(E.flag[k] & CF_VALID)) continue;
            const int e = MAXV * b + k, f = E.face[k], j = E.nbr[k];
            double nx = P.enx[e], ny = P.eny[e], S = P.es[e];   // the outward normal of a boundary face
            lc += (fabs(U * nx + V * ny) + cs) * S;
            double wj[5];
            if (j >= 0) {
#pragma unroll
                for (int k = 0; k < 4; k++) wj[k] = W[k * N + j];
            } else {
                ghost(ip, P.fbc[f], w, nx, ny, wj);
            }
            double dx = P.cf_dx[e], dy = P.cf_dy[e];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                double d = wj[k] - w[k];
                b1[k] += dx * d;
                b2[k] += dy * d;
                wmax[k] = fmax(wmax[k], wj[k]);
                wmin[k] = fmin(wmin[k], wj[k]);
            }
        }
    };
    const Entries E0 = entries(P, c);
    block(E0, c);
    const int ovf = next_block(P, E0);   // a polygon's overflow block, or -1
    if (ovf >= 0) block(entries(P, ovf), ovf);
    P.lamc[c] = lc;
    double L11 = P.lsinv[c], L12 = P.lsinv[N + c], L22 = P.lsinv[2 * N + c];
    double gx[4], gy[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        gx[k] = L11 * b1[k] + L12 * b2[k];
        gy[k] = L12 * b1[k] + L22 * b2[k];
    }
    double dUdy = (gy[1] - U * gy[0]) / r;
    double dVdx = (gx[2] - V * gx[0]) / r;
    P.vort[c] = fabs(dVdx - dUdy);
    if (P.limiter && P.is[inst].phi_frozen) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const double phi = P.phi[k * N + c];
            gx[k] *= phi;
            gy[k] *= phi;
        }
    } else if (P.limiter) {
        const int NB = P.nb;
        double nmax[4], nmin[4];
#pragma unroll
        for (int k = 0; k < 4; k++) { nmax[k] = -INFINITY; nmin[k] = INFINITY; }
        for (int b = c; b >= 0; b = (b == c) ? ovf : -1) {
            double vx[MAXV], vy[MAXV];
#pragma unroll
            for (int v = 0; v < MAXV; v++) { vx[v] = P.vtx[(2 * v) * NB + b]; vy[v] = P.vtx[(2 * v + 1) * NB + b]; }
#pragma unroll
            for (int k = 0; k < 4; k++) {
#pragma unroll
                for (int v = 0; v < MAXV; v++) {
                    double wv = w[k] + gx[k] * vx[v] + gy[k] * vy[v];
                    nmax[k] = fmax(nmax[k], wv);
                    nmin[k] = fmin(nmin[k], wv);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            double phi = 1.0;
            if (nmax[k] > w[k]) phi = fmin(phi, (wmax[k] - w[k]) / (nmax[k] - w[k]));
            if (nmin[k] < w[k]) phi = fmin(phi, (wmin[k] - w[k]) / (nmin[k] - w[k]));
            P.phi[k * N + c] = phi;
            gx[k] *= phi;
            gy[k] *= phi;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        P.grad[k * N + c] = gx[k];
        P.grad[(4 + k) * N + c] = gy[k];
    }
    return P.cfl_flux * P.area[c] / lc;
}

template <typename T, bool ONE>
__global__ __launch_bounds__(256) void k_prep(Params<T> P)
{
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    const int c = t < P.nc ? P.cperm[t] : P.nc;
    int inst = -1;
    double dt = INFINITY;
    if (c < P.nc) {
        inst = live_inst<ONE>(P, P.cinst, c);
        if (inst >= 0) dt = prep_cell(P, c, inst);
    }
    slot_update<true>(P.slot, SL_DTMIN, inst, dt);   // Eq.23: minimum over the instance's cells
}

// The Eq.23 time step of the lane's instance: the minimum over its slots.
// A wave whose lanes share one instance reads the 64 slots one per lane.
__device__ __forceinline__ double instance_dt(const unsigned long long *slot, int inst)
{
    unsigned long long act = __ballot(inst >= 0);
    if (act == 0ull) return 0.0;
    int i0 = __shfl(inst, __ffsll((long long)act) - 1);
    if (__all(inst < 0 || inst == i0)) return wave_min(slot_lane(slot, i0, SL_DTMIN));
    return inst >= 0 ? slots_min_serial(slot, inst, SL_DTMIN) : 0.0;
}

// rho > 0 and rho E - |rho U|^2 / (2 rho) > 0, the second tested as
// 2 rho (rho E) - |rho U|^2 > 0 (no divide)
__device__ __forceinline__ bool physical(const double *w)
{
    return w[0] > 0.0 && 2.0 * w[0] * w[3] - (w[1] * w[1] + w[2] * w[2]) > 0.0;
}

// One side of a face (side 0: the owner cell; side 1: the neighbour, or on
// a boundary face the ghost cell): reconstructed face state (Eq.10, the
// cell value where the reconstruction is not physical), slopes and
// cell-centre state rotated into the face frame (normal n out of the owner,
// tangent t = (-n_y, n_x)), the distance to the face and the side's
// spectral-radius and SA quantities.
struct FaceSide {
    double fw[4], gn[4], gt[4], fwc[4];
    double nut;               // nu~ of the cell-centre state
    double id;                // 1 / centroid-face distance (d_l or d_r)
    double ls, evr, nu, q;    // |V.n| + c, (mu + mu_t)/rho, nu, V.n
};
template <typename T>
__device__ __forceinline__ void face_side(const Params<T> &P, const InstParam &ip, const double *W, int f, int side,
                                          FaceSide &o)
{
    const int N = P.nc;
    const int l = P.fl[f], rr = P.fr[f];
    const bool bnd = rr < 0;
    const double nx = P.fnx[f], ny = P.fny[f], tx = -ny, ty = nx;
    // a ghost side starts from the owner's reconstruction
    const bool own = side == 0 || bnd;
    const int cm = own ? l : rr;
    const double *rv = own ? P.frl : P.frr;
    const double rx = rv[2 * f], ry = rv[2 * f + 1];
    double wm[5], WM[4], gx[4], gy[4];
#pragma unroll
    for (int k = 0; k < 5; k++) wm[k] = W[k * N + cm];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        gx[k] = P.grad[k * N + cm];
        gy[k] = P.grad[(4 + k) * N + cm];
        WM[k] = wm[k] + gx[k] * rx + gy[k] * ry;
    }
    if (!physical(WM)) {
#pragma unroll
        for (int k = 0; k < 4; k++) { WM[k] = wm[k]; gx[k] = gy[k] = 0.0; }
    }
    o.id = side ? P.fidr[f] : P.fidl[f];   // fidr = fidl on a boundary face
    const bool ghost_side = bnd && side == 1;
    const int bc = bnd ? P.fbc[f] : 0;
    // a moving wall is evaluated in its own frame from the owner's data, and
    // so is an isothermal static wall (u_w = 0): the reflected states let no
    // mass or energy through, the heat flux is added in wall_face_terms
    const bool moving = bc == BC_MOVING_WALL || (bc == BC_WALL && ip.tw > 0.0);
    auto rot = [&](const double *src, double *dst) {
        dst[0] = src[0];
        dst[1] = src[1] * nx + src[2] * ny;
        dst[2] = src[1] * tx + src[2] * ty;
        dst[3] = src[3];
    };
    // face-frame states: the side's own, or the owner's for a wall-frame face
    // (reflected below); otherwise the boundary map of the reconstructed
    // interior face state and of the interior cell centre
    if (!ghost_side || moving) {
        rot(WM, o.fw);
        rot(wm, o.fwc);
    }
    if (ghost_side) {
        double wg[5];
        if (!moving) {
            double tmp[5] = {WM[0], WM[1], WM[2], WM[3], wm[4]}, out[5];
            ghost(ip, bc, tmp, nx, ny, out);
            rot(out, o.fw);
        }
        ghost(ip, bc, wm, nx, ny, wg);
#pragma unroll
        for (int k = 0; k < 5; k++) wm[k] = wg[k];
        if (!moving) rot(wm, o.fwc);
    }
    {
        const double irm = frcp(wm[0]);
        o.q = (wm[1] * nx + wm[2] * ny) * irm;
        const double hm = half_inv_lam(wm, irm), c2 = GAMMA * hm;   // c^2 = gamma / (2 lambda)
        o.ls = fabs(o.q) + c2 * frsq(c2);
        const double mu = mu_hl(P.mu_law, ip, hm);
        double ev = mu;
        if (ip.sa && wm[4] > 0) ev += wm[0] * wm[4] * sa_fv1_f(wm[4] * wm[0] * frcp(mu));
        o.evr = ev * irm;
        o.nu = mu * irm;
        o.nut = wm[4];
    }
    {
        double tn[4], tt[4];
#pragma unroll
        for (int k = 0; k < 4; k++) { tn[k] = gx[k] * nx + gy[k] * ny; tt[k] = gx[k] * tx + gy[k] * ty; }
        rot(tn, o.gn);
        rot(tt, o.gt);
    }
    if (moving) {
        // the owner's face-frame state and slopes boosted by -u_w along the
        // face, (rho, m_n, m_t, E) -> (rho, m_n, m_t - u_w rho,
        // E - u_w m_t + u_w^2 rho / 2); the ghost side is then their point
        // reflection through a static no-slip wall
        const double uw = bc == BC_MOVING_WALL ? wall_speed(ip, nx, ny) : 0.0;
        double *bs[4] = {o.fw, o.fwc, o.gn, o.gt};
#pragma unroll
        for (int h = 0; h < 4; h++) {
            double *v = bs[h];
            v[3] = v[3] - uw * v[2] + 0.5 * uw * uw * v[0];
            v[2] = v[2] - uw * v[0];
        }
        if (ghost_side) {
            o.fw[1] = -o.fw[1]; o.fw[2] = -o.fw[2];
            o.fwc[1] = -o.fwc[1]; o.fwc[2] = -o.fwc[2];
            o.gn[0] = -o.gn[0]; o.gn[3] = -o.gn[3];
            o.gt[0] = -o.gt[0]; o.gt[3] = -o.gt[3];
        }
    } else if (ghost_side) {
        // ghost cell of a symmetry face = mirror image of the interior cell,
        // of a no-slip wall = its point reflection through the face
        // (bounce-back), slopes included: the normal derivative flips, the
        // boundary map acts on the face-frame momentum, and the wall also
        // flips the tangential derivative.  Free-stream and outflow ghosts
        // have zero slopes.
        if (bc == BC_SYMMETRY || bc == BC_WALL) {
            const double bt = (bc == BC_WALL) ? -1.0 : 1.0;
            const double n0 = o.gn[0], n1 = o.gn[1], n2 = o.gn[2], n3 = o.gn[3];
            const double t0 = o.gt[0], t1 = o.gt[1], t2 = o.gt[2], t3 = o.gt[3];
            o.gn[0] = -n0; o.gn[1] = n1; o.gn[2] = -bt * n2; o.gn[3] = -n3;
            o.gt[0] = bt * t0; o.gt[1] = -bt * t1; o.gt[2] = t2; o.gt[3] = bt * t3;
        } else {
#pragma unroll
            for (int k = 0; k < 4; k++) o.gn[k] = o.gt[k] = 0.0;
        }
    }
}

// Spectral radius of the face for the implicit operator and the SA face
// terms (Eq.28-30) from the two sides' quantities (l the owner, r the
// neighbour or ghost).
struct FaceTerms {
    double lam, saf, sag, sak;   // saf = (-F_inv + F_vis) S, sag = g S out of the owner, sak = k S / |r.n|
};
template <typename T>
__device__ __forceinline__ FaceTerms face_implicit_terms(const Params<T> &P, const InstParam &ip, int f, double lsl,
                                                         double lsr, double evl, double evr, double nul, double nur,
                                                         double ti, double tj, double ql, double qr)
{
    const double irn = P.firn[f], S = P.flen[f];
    FaceTerms o{fmax(lsl, lsr), 0.0, 0.0, 0.0};
    if (P.visc_sr) o.lam += (evl + evr) * irn;
    if (ip.sa) {
        double g = (tj - ti) * irn;
        double Finv = 0.5 * (ql + fabs(ql)) * ti + 0.5 * (qr - fabs(qr)) * tj;
        double kf = (0.5 / SA_SIGMA) * ((nul + nur) + (1.0 + SA_CB2) * (ti + tj));
        o.saf = (kf * g - Finv) * S;
        o.sag = g * S;
        o.sak = kf * S * irn;
    }
    return o;
}

// Two values into a face record with one 16-byte store (k even).
__device__ __forceinline__ void rec_store2(double *r, int k, double a, double b)
{
    *reinterpret_cast<double2 *>(r + k) = make_double2(a, b);
}
// The face terms into the face record and the packed arrays, stored as soon
// as they are formed so that they do not stay live across the flux.  half
// 0: lam and saf, half 1: sag and sak, -1: all four (the one-lane kernel).
template <typename T>
__device__ __forceinline__ void store_terms(const Params<T> &P, const InstParam &ip, int f, const FaceTerms &t,
                                            int half)
{
    double *r = P.frec + FR_STRIDE * (size_t)f;
    if (half <= 0) {
        rec_store2(r, FR_LAM, t.lam, t.saf);
        P.flam[f] = t.lam;
    }
    if (half != 0) {
        rec_store2(r, FR_SAG, t.sag, t.sak);
        if (ip.sa) P.fsak[f] = t.sak;
    }
}

// face-frame flux integrated over [0, dt] -> F S / dt in the global frame
__device__ __forceinline__ void flux_global(const double *Fr, double dt, double nx, double ny, double S, double *g)
{
    const double tx = -ny, ty = nx, idt = frcp(dt);
    const double Fn = Fr[1] * idt, Ft = Fr[2] * idt;
    g[0] = Fr[0] * idt * S;
    g[1] = (Fn * nx + Ft * tx) * S;
    g[2] = (Fn * ny + Ft * ty) * S;
    g[3] = Fr[3] * idt * S;
}

// Per face, one lane: both sides, the GKS flux, the implicit terms.
template <typename T>
__device__ __forceinline__ void flux_face(const Params<T> &P, int f, int inst, double dt)
{
    const InstParam &ip = P.ip[inst];
    const double *W = cur_state(P, inst);
    FaceSide L, R;
    face_side(P, ip, W, f, 0, L);
    face_side(P, ip, W, f, 1, R);
    store_terms(P, ip, f, face_implicit_terms(P, ip, f, L.ls, R.ls, L.evr, R.evr, L.nu, R.nu, L.nut, R.nut, L.q, R.q),
                -1);
    const double nutf = fmax(0.5 * add_sides(L.nut, R.nut), 0.0);
    double acc[24], accr[24];
    side_terms(1.0, L.fw, L.gn, L.gt, acc);
    side_terms(-1.0, R.fw, R.gn, R.gt, accr);
#pragma unroll
    for (int k = 0; k < 24; k++) acc[k] = add_sides(acc[k], accr[k]);
    // optional collision-time term from the pressure jump across the face
    double jump = 0.0;
    if (P.tau_jump) {
        const double pl = L.fw[3] - 0.5 * (L.fw[1] * L.fw[1] + L.fw[2] * L.fw[2]) / L.fw[0];
        const double pr = R.fw[3] - 0.5 * (R.fw[1] * R.fw[1] + R.fw[2] * R.fw[2]) / R.fw[0];
        jump = fabs(pl - pr) / (pl + pr);
    }
    GksEq q;
    gks_eq(P, ip, acc, dt, nutf, jump, q);
    double q2[4], f2[4], q2r[4], f2r[4], gts[4];
    gks_half(q, 1.0, acc, L.fwc, L.id, q2, f2);
    gks_half(q, -1.0, acc, R.fwc, R.id, q2r, f2r);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        q2[k] = add_sides(q2[k], q2r[k]);
        f2[k] = add_sides(f2[k], f2r[k]);
        gts[k] = add_sides(L.gt[k], R.gt[k]);
    }
    double Fr[4], g[4];
    gks_finish(q, acc, q2, f2, gts, dt, Fr);
    flux_global(Fr, dt, P.fnx[f], P.fny[f], P.flen[f], g);
    double *r = P.frec + FR_STRIDE * (size_t)f;
    rec_store2(r, FR_F0, g[0], g[1]);
    rec_store2(r, FR_F2, g[2], g[3]);
}

// Per face, on a pair of lanes (side 0 the owner, side 1 the neighbour or
// ghost): each lane builds its side and integrates its half space; the sums
// of the two halves are formed on both lanes (a + b is the same number in
// either order) and the equilibrium part is evaluated on both.  Both lanes
// of a pair call this together.
template <typename T>
__device__ __forceinline__ void flux_face_pair(const Params<T> &P, int f, int side, int inst, double dt)
{
    const InstParam &ip = P.ip[inst];
    const double *W = cur_state(P, inst);
    FaceSide M;
    face_side(P, ip, W, f, side, M);
    {
        // both lanes form the face terms (owner's values first) and each
        // stores half of them
        const double ls_o = pair_other(M.ls), evr_o = pair_other(M.evr), nu_o = pair_other(M.nu);
        const double t_o = pair_other(M.nut), q_o = pair_other(M.q);
        const double lsl = side ? ls_o : M.ls, lsr = side ? M.ls : ls_o;
        const double evl = side ? evr_o : M.evr, evr = side ? M.evr : evr_o;
        const double nul = side ? nu_o : M.nu, nur = side ? M.nu : nu_o;
        const double til = side ? t_o : M.nut, tir = side ? M.nut : t_o;
        const double ql = side ? q_o : M.q, qr = side ? M.q : q_o;
        store_terms(P, ip, f, face_implicit_terms(P, ip, f, lsl, lsr, evl, evr, nul, nur, til, tir, ql, qr), side);
    }
    const double nutf = fmax(0.5 * add_sides(M.nut, pair_other(M.nut)), 0.0);
    const double sgn = side ? -1.0 : 1.0;
    double acc[24];
    side_terms(sgn, M.fw, M.gn, M.gt, acc);
#pragma unroll
    for (int k = 0; k < 24; k++) acc[k] = add_sides(acc[k], pair_other(acc[k]));
    double jump = 0.0;
    if (P.tau_jump) {
        const double ps = M.fw[3] - 0.5 * (M.fw[1] * M.fw[1] + M.fw[2] * M.fw[2]) / M.fw[0];
        const double po = pair_other(ps);
        const double pl = side ? po : ps, pr = side ? ps : po;
        jump = fabs(pl - pr) / (pl + pr);
    }
    GksEq q;
    gks_eq(P, ip, acc, dt, nutf, jump, q);
    double q2[4], f2[4], gts[4];
    gks_half(q, sgn, acc, M.fwc, M.id, q2, f2);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        q2[k] = add_sides(q2[k], pair_other(q2[k]));
        f2[k] = add_sides(f2[k], pair_other(f2[k]));
        gts[k] = add_sides(M.gt[k], pair_other(M.gt[k]));
    }
    double Fr[4], g[4];
    gks_finish(q, acc, q2, f2, gts, dt, Fr);
    flux_global(Fr, dt, P.fnx[f], P.fny[f], P.flen[f], g);
    // each lane writes two of the four components, one 16-byte store
    rec_store2(P.frec + FR_STRIDE * (size_t)f, side ? FR_F2 : FR_F0, side ? g[2] : g[0], side ? g[3] : g[1]);
}

// one lane per face
template <typename T, bool ONE>
__global__ __launch_bounds__(256) void k_flux(Params<T> P)
{
    const int f = xcd_block() * blockDim.x + threadIdx.x;
    int inst = -1;
    if (f < P.nf) inst = live_inst<ONE>(P, P.finst, f);
    double dt = instance_dt(P.slot, inst);
    if (inst < 0) return;
    flux_face(P, f, inst, dt);
}

// two lanes per face
template <typename T, bool ONE>
__global__ __launch_bounds__(256) void k_flux2(Params<T> P)
{
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    const int f = t >> 1, side = t & 1;
    int inst = -1;
    if (f < P.nf) inst = live_inst<ONE>(P, P.finst, f);
    double dt = instance_dt(P.slot, inst);
    if (inst < 0) return;   // both lanes of a pair leave together
    flux_face_pair(P, f, side, inst, dt);
}

// The flux of a no-slip wall face as stored by the flux kernels (g = F S in
// the global frame) completed here, where the cell's state is at hand: a
// moving wall's flux goes from the wall's frame back to the mesh frame
// (F_E += u_w F_t + u_w^2 F_rho / 2, F_t += u_w F_rho), and an isothermal
// wall adds the heat flux mu c_p (T_c - T_w) / d_l S of the BGK model
// (Pr = 1, c_p = gamma / (gamma - 1) in units of R).  Kept out of the flux
// kernels, whose register budget sets their occupancy.
template <typename T>
__device__ __forceinline__ void wall_face_terms(const Params<T> &P, const InstParam &ip, const double *w, int f,
                                                double *g)
{
    const int bc = P.fbc[f];
    if (bc != BC_WALL && bc != BC_MOVING_WALL) return;
    if (bc == BC_MOVING_WALL) {
        const double nx = P.fnx[f], ny = P.fny[f], uw = wall_speed(ip, nx, ny);
        const double ft = -g[1] * ny + g[2] * nx;
        g[3] += uw * ft + 0.5 * uw * uw * g[0];
        g[1] += uw * g[0] * (-ny);
        g[2] += uw * g[0] * nx;
    }
    if (ip.tw > 0.0) {
        const double lc = lam_of(w);
        const double kappa = mu_lam(P.mu_law, ip, lc) * (GAMMA / (GAMMA - 1.0));
        g[3] += kappa * (0.5 / lc - ip.tw) * P.fidl[f] * P.flen[f];
    }
}

// Per cell: residual M (Eq.16) as the signed sum of its face fluxes, the
// LU-SGS diagonal pieces, the SA residual and diagonal (Eq.27-32), the
// squares for the L2 norms and the max norm.
template <typename T>
__device__ __forceinline__ double gather_cell(const Params<T> &P, int c, int inst)
{
    const int N = P.nc;
    const InstParam &ip = P.ip[inst];
    const double *W = cur_state(P, inst);
    double m[4] = {0, 0, 0, 0}, ls = 0.0, saR = 0.0, sagS = 0.0, sad = 0.0;
    double w[5];
#pragma unroll
    for (int k = 0; k < 5; k++) w[k] = W[k * N + c];
    double nuc = P.nu[c];
    auto block = [&](const Entries &E, int b) {
#pragma unroll
        for (int k = 0; k < MAXV; k++) {
            if (!(E.flag[k] & CF_VALID)) continue;
            const int e = MAXV * b + k, f = E.face[k];
            double sg = (E.flag[k] & CF_OWNER) ? 1.0 : -1.0;
            const double *r = P.frec + FR_STRIDE * (size_t)f;
            double g[4] = {r[FR_F0], r[FR_F1], r[FR_F2], r[FR_F3]};
            if (E.nbr[k] < 0) wall_face_terms(P, ip, w, f, g);
#pragma unroll
            for (int k = 0; k < 4; k++) m[k] -= sg * g[k];
            double S = P.es[e];
            ls += r[FR_LAM] * S;
            if (ip.sa) {
                saR += sg * r[FR_SAF];
                sagS += sg * r[FR_SAG];
                double qc = (w[1] * P.enx[e] + w[2] * P.eny[e]) / w[0];   // the normal out of the cell
                sad += 0.5 * (qc + fabs(qc)) * S + r[FR_SAK];
            }
        }
    };
    const Entries E0 = entries(P, c);
    block(E0, c);
    const int ovf = next_block(P, E0);
    if (ovf >= 0) block(entries(P, ovf), ovf);
#pragma unroll
    for (int k = 0; k < 4; k++) P.M[k * N + c] = m[k];
    P.lsum[c] = 0.5 * ls;
    const int pos = P.ipos[c];
    P.r2[pos] = m[0] * m[0];
    if (ip.sa) {
        double Sr, jd;
        sa_source(w[4], nuc, P.dwall[c], P.vort[c], Sr, jd);
        double a = P.area[c];
        double rsa = saR - (SA_CB2 / SA_SIGMA) * w[4] * sagS + a * Sr;
        P.M[4 * N + c] = rsa;
        P.sadiag[c] = sad + a * jd;
        P.r2[N + pos] = rsa * rsa;
    } else {
        P.M[4 * N + c] = 0.0;
        P.r2[N + pos] = 0.0;
    }
    return fmax(fmax(fabs(m[0]), fabs(m[1])), fmax(fabs(m[2]), fabs(m[3])));
}

template <typename T, bool ONE>
__global__ __launch_bounds__(256) void k_gather(Params<T> P)
{
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    const int c = t < P.nc ? P.cperm[t] : P.nc;
    int inst = -1;
    double rinf = 0.0;
    if (c < P.nc) {
        inst = live_inst<ONE>(P, P.cinst, c);
        if (inst >= 0) rinf = gather_cell(P, c, inst);
    }
    slot_update<false>(P.slot, SL_RESINF, inst, rinf);
}

// Sum over the wave by butterfly: every lane ends with the same value (each
// step adds the same two numbers on both lanes), in a fixed order.
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 1; o < warpSize; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

// Norm partial sums: block (i, b) sums slice b (NORM_SLICE squares; the
// slices past the instance's end are empty) of instance i's squares
// (contiguous, instance-grouped) in a fixed order, so the L2 norms are
// deterministic without float atomics and the same whatever the other
// instances of the context; k_commit adds the rb partial sums.
template <typename T>
__device__ __forceinline__ void norm_partial(const Params<T> &P, int blk)
{
    __shared__ double a[256], b[256];
    int i = blk / P.rb, part = blk % P.rb;
    int lo = P.ioff[i], n = P.ioff[i + 1] - lo;
    int s0 = lo + min(n, part * NORM_SLICE), s1 = lo + min(n, (part + 1) * NORM_SLICE);
    double x = 0.0, y = 0.0;
    const double *r2a = P.r2, *r2b = P.r2 + P.nc;
#pragma unroll 4
    for (int k = s0 + (int)threadIdx.x; k < s1; k += 256) {
        x += r2a[k];
        y += r2b[k];
    }
    a[threadIdx.x] = x;
    b[threadIdx.x] = y;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) { a[threadIdx.x] += a[threadIdx.x + h]; b[threadIdx.x] += b[threadIdx.x + h]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        P.ipart[2 * blk] = a[0];
        P.ipart[2 * blk + 1] = b[0];
    }
}

// Blocks [0, ninst rb): the norm partial sums.  Block ninst rb + i, first
// wave: the Eq.23 time step the flux used, the max norm, the Eq.25 CFL law
// (the L2 norms are not needed before the commit), history entry `it` of
// the chunk.
template <typename T>
__global__ __launch_bounds__(256) void k_reduce(Params<T> P, int it)
{
    if ((int)blockIdx.x < P.ninst * P.rb) {
        norm_partial(P, blockIdx.x);
        return;
    }
    const int i = blockIdx.x - P.ninst * P.rb, lane = threadIdx.x;
    if (lane >= 64) return;
    InstScalars *s = &P.is[i];
    if (s->halt) return;
    double dt = wave_min(slot_lane(P.slot, i, SL_DTMIN));
    double rinf = wave_max(slot_lane(P.slot, i, SL_RESINF));
    *slot_at(P.slot, i, SL_RESINF, lane) = 0ull;
    if (lane != 0) return;
    s->dt = dt;
    if (s->ncommit == 0) {
        s->cfl = P.cfl_init;
    } else if (P.cfl_mode == 0) {
        double cf = s->cfl * s->res_inf_prev / rinf;
        if (!(cf >= P.cfl_min)) cf = P.cfl_min;
        if (cf > P.cfl_max) cf = P.cfl_max;
        s->cfl = cf;
    }
    s->res_inf_prev = rinf;
    s->res_inf = rinf;
    if (it < P.hist_cap) {
        double *e = P.hist + (size_t)HIST_W * ((size_t)it * P.ninst + i);
        e[1] = rinf; e[2] = s->cfl; e[3] = dt;
    }
}

// Accumulation of the sweeps' neighbour terms, never fused with the
// product that formed a term: the one-lane and the quad-lane sweeps then
// form the same numbers.
template <typename V>
__device__ __forceinline__ V acc_sub(V a, V b)
{
#pragma clang fp contract(off)
    return a - b;
}
template <typename V>
__device__ __forceinline__ V acc_add(V a, V b)
{
#pragma clang fp contract(off)
    return a + b;
}

// Value of lane K of the lane's quad (a DPP quad permutation; every lane of
// the quad must be active).
template <int K>
__device__ __forceinline__ int quad_get(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, K * 0x55, 0xf, 0xf, false);
}
template <int K>
__device__ __forceinline__ float quad_get(float v)
{
    return __int_as_float(quad_get<K>(__float_as_int(v)));
}
template <int K>
__device__ __forceinline__ double quad_get(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = quad_get<K>((int)(b & 0xffffffffll)), hi = quad_get<K>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// a -= t_0, t_1, t_2, t_3 (SUB) or a += them, in lane order, t_k the value
// on lane k of the quad: the order of the one-lane loop over four entries
template <bool SUB, typename V>
__device__ __forceinline__ V quad_fold(V a, V t)
{
    const V t0 = quad_get<0>(t), t1 = quad_get<1>(t), t2 = quad_get<2>(t), t3 = quad_get<3>(t);
    if (SUB) return acc_sub(acc_sub(acc_sub(acc_sub(a, t0), t1), t2), t3);
    return acc_add(acc_add(acc_add(acc_add(a, t0), t1), t2), t3);
}

// ---- Roe-matrix LU-SGS operator (option lusgs_op = 1 or 2) ----
// The dissipation of the first-order Roe flux (Eq.18) in place of the
// scalar spectral radius of Eq.20: |A| = R |Lambda| L of the Euler flux
// Jacobian at the Roe average of the two cell-centre states.  The magnitudes
// of the eigenvalues s = q - c, q, q, q + c: option 1, |s| held at least at
// ROE_DELTA c; option 2, the mean of |u| for u ~ N(s, RT), RT = c^2 / gamma,
// s erf(s / sqrt(2RT)) + sqrt(2RT / pi) exp(-s^2 / (2RT)) (the spread a
// Maxwellian gives each wave at the interface).

constexpr double ROE_DELTA = 0.1;

// Roe average of states a (the cell) and b (the neighbour or ghost) for the
// normal n out of the cell; smax = max(|q_a| + c_a, |q_b| + c_b), the
// inviscid part of the face's spectral radius; m0, m1, m3 the magnitudes of
// the eigenvalues q - c, q, q + c
struct RoeAvg {
    double u, v, H, k, c, q, qt, smax, m0, m1, m3;
};

__device__ __forceinline__ double kin_mag(double s, double rt2)
{
    return s * erf(s / sqrt(rt2)) + sqrt(rt2 * (1.0 / M_PI)) * exp(-s * s / rt2);
}

__device__ __forceinline__ RoeAvg roe_avg(const double *a, const double *b, double nx, double ny, bool kin)
{
    const double g1 = GAMMA - 1.0;
    const double ra = a[0], rb = b[0];
    const double ua = a[1] / ra, va = a[2] / ra, ub = b[1] / rb, vb = b[2] / rb;
    const double pa = g1 * (a[3] - 0.5 * (a[1] * ua + a[2] * va)), pb = g1 * (b[3] - 0.5 * (b[1] * ub + b[2] * vb));
    const double sa = sqrt(ra), sb = sqrt(rb), iw = 1.0 / (sa + sb);
    RoeAvg R;
    R.u = (sa * ua + sb * ub) * iw;
    R.v = (sa * va + sb * vb) * iw;
    R.H = (sa * (a[3] + pa) / ra + sb * (b[3] + pb) / rb) * iw;
    R.k = 0.5 * (R.u * R.u + R.v * R.v);
    R.c = sqrt(g1 * (R.H - R.k));
    R.q = R.u * nx + R.v * ny;
    R.qt = -R.u * ny + R.v * nx;
    R.smax = fmax(fabs(ua * nx + va * ny) + sqrt(GAMMA * pa / ra), fabs(ub * nx + vb * ny) + sqrt(GAMMA * pb / rb));
    if (kin) {
        const double rt2 = 2.0 * R.c * R.c / GAMMA;   // 2RT
        R.m0 = kin_mag(R.q - R.c, rt2);
        R.m1 = kin_mag(R.q, rt2);
        R.m3 = kin_mag(R.q + R.c, rt2);
    } else {
        const double fl = ROE_DELTA * R.c;
        R.m0 = fmax(fabs(R.q - R.c), fl);
        R.m1 = fmax(fabs(R.q), fl);
        R.m3 = fmax(fabs(R.q + R.c), fl);
    }
    return R;
}

// out = |A| d by the wave decomposition: wave strengths alpha = L d (a
// pressure part dp / c^2 and a normal-velocity part), each scaled by its
// eigenvalue magnitude, summed over the right eigenvectors
__device__ __forceinline__ void roe_apply(const RoeAvg &R, double nx, double ny, const double *d, double *out)
{
    const double ic = 1.0 / R.c, g1c2 = (GAMMA - 1.0) * ic * ic;
    const double dpc = g1c2 * (R.k * d[0] - R.u * d[1] - R.v * d[2] + d[3]);
    const double dun = (-R.q * d[0] + nx * d[1] + ny * d[2]) * ic;
    const double a0 = 0.5 * (dpc - dun) * R.m0;
    const double a3 = 0.5 * (dpc + dun) * R.m3;
    const double a1 = (d[0] - dpc) * R.m1;
    const double a2 = (-R.qt * d[0] - ny * d[1] + nx * d[2]) * R.m1;
    out[0] = a0 + a1 + a3;
    out[1] = a0 * (R.u - R.c * nx) + a1 * R.u - a2 * ny + a3 * (R.u + R.c * nx);
    out[2] = a0 * (R.v - R.c * ny) + a1 * R.v + a2 * nx + a3 * (R.v + R.c * ny);
    out[3] = a0 * (R.H - R.q * R.c) + a1 * R.k + a2 * R.qt + a3 * (R.H + R.q * R.c);
}

// inverse of a 4x4 matrix (row-major) by cofactors: the 2x2 minors of the
// top two rows (s) and of the bottom two rows (c) give the determinant by
// Laplace expansion and every cofactor
__device__ __forceinline__ void inv4x4(const double *a, double *b)
{
    const double s0 = a[0] * a[5] - a[4] * a[1], s1 = a[0] * a[6] - a[4] * a[2], s2 = a[0] * a[7] - a[4] * a[3];
    const double s3 = a[1] * a[6] - a[5] * a[2], s4 = a[1] * a[7] - a[5] * a[3], s5 = a[2] * a[7] - a[6] * a[3];
    const double c5 = a[10] * a[15] - a[14] * a[11], c4 = a[9] * a[15] - a[13] * a[11];
    const double c3 = a[9] * a[14] - a[13] * a[10], c2 = a[8] * a[15] - a[12] * a[11];
    const double c1 = a[8] * a[14] - a[12] * a[10], c0 = a[8] * a[13] - a[12] * a[9];
    const double id = 1.0 / (s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0);
    b[0] = (a[5] * c5 - a[6] * c4 + a[7] * c3) * id;
    b[1] = (-a[1] * c5 + a[2] * c4 - a[3] * c3) * id;
    b[2] = (a[13] * s5 - a[14] * s4 + a[15] * s3) * id;
    b[3] = (-a[9] * s5 + a[10] * s4 - a[11] * s3) * id;
    b[4] = (-a[4] * c5 + a[6] * c2 - a[7] * c1) * id;
    b[5] = (a[0] * c5 - a[2] * c2 + a[3] * c1) * id;
    b[6] = (-a[12] * s5 + a[14] * s2 - a[15] * s1) * id;
    b[7] = (a[8] * s5 - a[10] * s2 + a[11] * s1) * id;
    b[8] = (a[4] * c4 - a[5] * c2 + a[7] * c0) * id;
    b[9] = (-a[0] * c4 + a[1] * c2 - a[3] * c0) * id;
    b[10] = (a[12] * s4 - a[13] * s2 + a[15] * s0) * id;
    b[11] = (-a[8] * s4 + a[9] * s2 - a[11] * s0) * id;
    b[12] = (-a[4] * c3 + a[5] * c1 - a[6] * c0) * id;
    b[13] = (a[0] * c3 - a[1] * c1 + a[2] * c0) * id;
    b[14] = (-a[12] * s3 + a[13] * s1 - a[14] * s0) * id;
    b[15] = (a[8] * s3 - a[9] * s1 + a[10] * s0) * id;
}

// Per cell, once the CFL number of the iteration is known: the LU-SGS
// diagonal block D = (Omega/dt) I + 1/2 sum (|A_f| + (lambda_f - smax_f) I) S_f
// (lambda_f - smax_f, the viscous part of the spectral radius, enters as
// before; 1/2 sum lambda_f S_f is lsum), inverted and stored for the sweeps.
// A face to another sweep block keeps lambda_f I: the block sweeps leave its
// coupling out, and the scalar operator's larger diagonal keeps that
// omission dominated (with |A| there the block iteration stalls).
template <typename T, bool ONE>
__global__ __launch_bounds__(256) void k_roe_diag(Params<T> P)
{
    const int N = P.nc;
    const int c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= N) return;
    const int inst = live_inst<ONE>(P, P.cinst, c);
    if (inst < 0) return;
    const InstParam &ip = P.ip[inst];
    const double *W = cur_state(P, inst);
    double w[5];
#pragma unroll
    for (int k = 0; k < 5; k++) w[k] = W[k * N + c];
    double a[16];
#pragma unroll
    for (int k = 0; k < 16; k++) a[k] = 0.0;
    auto block = [&](const Entries &E, int b) {
#pragma unroll
        for (int k = 0; k < MAXV; k++) {
            if (!(E.flag[k] & CF_VALID) || (E.flag[k] & CF_OTHER)) continue;
            const int e = MAXV * b + k, f = E.face[k], j = E.nbr[k];
            const double nx = P.enx[e], ny = P.eny[e], hS = 0.5 * P.es[e];
            double wj[5];
            if (j >= 0) {
#pragma unroll
                for (int m = 0; m < 5; m++) wj[m] = W[m * N + j];
            } else {
                ghost(ip, P.fbc[f], w, nx, ny, wj);
            }
            const RoeAvg R = roe_avg(w, wj, nx, ny, P.roe_kin);
#pragma unroll
            for (int col = 0; col < 4; col++) {
                double d[4] = {0.0, 0.0, 0.0, 0.0}, o[4];
                d[col] = 1.0;
                roe_apply(R, nx, ny, d, o);
#pragma unroll
                for (int r = 0; r < 4; r++) a[4 * r + col] += hS * o[r];
            }
#pragma unroll
            for (int r = 0; r < 4; r++) a[5 * r] -= hS * R.smax;
        }
    };
    const Entries E0 = entries(P, c);
    block(E0, c);
    const int ovf = next_block(P, E0);
    if (ovf >= 0) block(entries(P, ovf), ovf);
    const double dg = P.lamc[c] / P.is[inst].cfl + P.lsum[c];
#pragma unroll
    for (int r = 0; r < 4; r++) a[5 * r] += dg;
    double b[16];
    inv4x4(a, b);
#pragma unroll
    for (int k = 0; k < 16; k++) P.dinv[k * N + c] = T(b[k]);
}

// y = D_c^-1 x with the stored inverse block (fixed order of operations)
template <typename T>
__device__ __forceinline__ void dinv_apply(const Params<T> &P, int c, const T *x, T *y)
{
    const int N = P.nc;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        T s = T(P.dinv[(4 * r) * N + c]) * x[0];
        s = fma(T(P.dinv[(4 * r + 1) * N + c]), x[1], s);
        s = fma(T(P.dinv[(4 * r + 2) * N + c]), x[2], s);
        y[r] = fma(T(P.dinv[(4 * r + 3) * N + c]), x[3], s);
    }
}

// Forward-sweep increment dW*_j of a cell of the first wavefront: it has no
// lower neighbours, so Eq.22 reduces to dW*_j = D_j^-1 M_j (the expressions
// of sweep_cell with nothing subtracted, hence the same numbers).  Formed
// where it is needed instead of in a launch of its own.
template <typename T, bool ROE>
__device__ __forceinline__ void first_front_incr(const Params<T> &P, const InstParam &ip, int j, T cfl, T *d)
{
    const int N = P.nc;
    const T odt = T(P.lamc[j]) / cfl;
    if (ROE) {
        T m[4];
#pragma unroll
        for (int k = 0; k < 4; k++) m[k] = T(P.M[k * N + j]);
        dinv_apply(P, j, m, d);
    } else {
        const T iD = T(1) / (odt + T(P.lsum[j]));
#pragma unroll
        for (int k = 0; k < 4; k++) d[k] = T(P.M[k * N + j]) * iD;
    }
    d[4] = ip.sa ? T(P.M[4 * N + j]) / (odt + T(P.sadiag[j])) : T(0);
}

// Neighbour term of one cell-face entry in the LU-SGS sweeps (Eq.22 and
// Eq.31-32): t[0..3] = (J(W_j, n) dW_j - lam dW_j) S / 2 with n pointing out
// of the cell (the Roe operator: |A| + (lam - smax) I in place of lam,
// except across sweep blocks, cross), t[4] = the SA off-diagonal coefficient
// times dnu~_j, dW_j read from dsrc.  j < 0: the ghost cell, whose increment follows from the cell's
// own dW* (Sec. 2.5).  Neighbours j < lev1 belong to the first wavefront,
// whose forward increments are not stored (first_front_incr).
template <typename T, bool ROE>
__device__ __forceinline__ void sweep_term(const Params<T> &P, const InstParam &ip, const double *W,
                                           const double *w, int f, int e, int j, const T *dws, T cfl, int lev1,
                                           T *t, const T *dsrc, bool cross = false)
{
    const int N = P.nc;
    double nx = P.enx[e], ny = P.eny[e];   // out of the cell
    T S = T(P.es[e]), lam = T(P.flam[f]);
    double wj[5];
    T dj[5];
    if (j >= 0) {
#pragma unroll
        for (int k = 0; k < 5; k++) wj[k] = W[k * N + j];
        if (j < lev1) {
            first_front_incr<T, ROE>(P, ip, j, cfl, dj);
        } else {
#pragma unroll
            for (int k = 0; k < 5; k++) dj[k] = dsrc[k * N + j];
        }
    } else {
        ghost(ip, P.fbc[f], w, nx, ny, wj);
        ghost_incr<T>(P.fbc[f], dws, T(nx), T(ny), T(wall_speed(ip, nx, ny)), dj);
    }
    T wjt[4] = {T(wj[0]), T(wj[1]), T(wj[2]), T(wj[3])};
    T jv[4];
    jac_vec<T>(wjt, T(nx), T(ny), dj, jv);
    T h = T(0.5) * S;
    if (ROE && !cross) {
        // (|A| + (lambda - smax) I) dW_j: the Roe matrix plus the viscous
        // part of the spectral radius
        const RoeAvg R = roe_avg(w, wj, nx, ny, P.roe_kin);
        const double dd[4] = {double(dj[0]), double(dj[1]), double(dj[2]), double(dj[3])};
        double ad[4];
        roe_apply(R, nx, ny, dd, ad);
        const T lv = lam - T(R.smax);
#pragma unroll
        for (int k = 0; k < 4; k++) t[k] = h * (jv[k] - lv * dj[k] - T(ad[k]));
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++) t[k] = h * (jv[k] - lam * dj[k]);
    }
    t[4] = T(0);
    if (ip.sa) {
        double qj = (wj[1] * nx + wj[2] * ny) / wj[0];
        double off = -0.5 * (qj - fabs(qj)) * P.es[e] + P.fsak[f];
        t[4] = T(off) * dj[4];
    }
}

// sweep modes
enum { SW_FWD = 0, SW_BWD = 1, SW_TOP = 2, SW_BWD_ONLY = 3 };

// W^{n+1} = W^n + dW (Eq.17) into the instance's other state buffer, nu~
// clipped at 0; flags a non-physical result; returns the Eq.40 ratio
// |dW| / |W| over the four flow variables.
template <typename T>
__device__ __forceinline__ double apply_update(const Params<T> &P, int c, int inst, const double *w, const double *d)
{
    const int N = P.nc;
    double *Wn = (P.is[inst].ncommit & 1) ? P.Wa : P.Wb;
    double wn[4], num = 0.0, den = 0.0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        num += d[k] * d[k];
        den += w[k] * w[k];
        wn[k] = w[k] + d[k];
        Wn[k * N + c] = wn[k];
    }
    double tt = w[4];
    if (P.ip[inst].sa) tt = fmax(tt + d[4], 0.0);
    Wn[4 * N + c] = tt;
    double p = wn[3] - 0.5 * (wn[1] * wn[1] + wn[2] * wn[2]) / wn[0];
    if (!(wn[0] > 0.0) || !(p > 0.0) || !isfinite(tt) || !isfinite(p)) atomicOr(&P.is[inst].bad, 1);
    double r = sqrt(num / den);
    return isfinite(r) ? r : 0.0;
}

// Explicit step (Eq.15) with the local time step dt_i = CFL Omega_i /
// (Lambda_c)_i of Eq.21/23: dW_i = dt_i M_i / Omega_i = CFL M_i / (Lambda_c)_i,
// the SA variable the same way with its right-hand side.
template <typename T, bool ONE>
__global__ __launch_bounds__(256) void k_explicit(Params<T> P)
{
    const int N = P.nc;
    int c = xcd_block() * blockDim.x + threadIdx.x;
    int inst = -1;
    double e = 0.0;
    if (c < N) {
        inst = live_inst<ONE>(P, P.cinst, c);
        if (inst >= 0) {
            const double *W = cur_state(P, inst);
            double w[5], d[5];
#pragma unroll
            for (int k = 0; k < 5; k++) w[k] = W[k * N + c];
            const double kc = P.is[inst].cfl / P.lamc[c];
#pragma unroll
            for (int k = 0; k < 4; k++) d[k] = kc * P.M[k * N + c];
            d[4] = P.ip[inst].sa ? kc * P.M[4 * N + c] : 0.0;
            e = apply_update(P, c, inst, w, d);
        }
    }
    slot_update<false>(P.slot, SL_E40, inst, e);
}

// One wavefront of the LU-SGS sweeps (Eq.22); the cells of a wavefront are
// mutually independent.  Forward:
//   dW*_i = D^-1 [M_i - sum_{j<i} (J(W_j, n_ij) dW*_j - lam_ij dW*_j) S_ij / 2];
// backward, in place:
//   dW_i = dW*_i - D^-1 sum_{j>i} (J(W_j, n_ij) dW_j - lam_ij dW_j) S_ij / 2,
// boundary ghosts counted as upper neighbours with the ghost increments of
// Sec. 2.5 taken from dW*_i.  The SA equation (Eq.31-32) is swept alongside.
// SW_TOP does both for the last wavefront: a neighbour j > i of a cell i
// always lies in a later wavefront, so the cells of the last one have only
// ghosts above them and their backward step needs nothing from other cells.
// The backward step also applies W^{n+1} = W^n + dW (Eq.17) into the
// instance's other state buffer (nu~ clipped at 0), flags a non-physical
// result and returns the Eq.40 ratio; SW_BWD_ONLY leaves the update to
// k_update.  inst = -1 for a frozen instance.
template <typename T, int MODE, bool ONE, bool ROE>
__device__ __forceinline__ double sweep_cell(const Params<T> &P, int c, int &inst)
{
    const int N = P.nc;
    inst = live_inst<ONE>(P, P.cinst, c);
    if (inst < 0) return 0.0;
    const InstScalars &sc = P.is[inst];
    const InstParam &ip = P.ip[inst];
    const double *W = cur_state(P, inst);
    const T cfl = T(sc.cfl);
    double w[5];
#pragma unroll
    for (int k = 0; k < 5; k++) w[k] = W[k * N + c];
    const Entries E0 = entries(P, c);
    const int ovf = next_block(P, E0);   // a polygon's overflow block, or -1
    const T odt = T(P.lamc[c]) / cfl;   // Omega / dt_imp with dt_imp = CFL Omega / Lambda_c (Eq.24)
    const T D = odt + T(P.lsum[c]);
    T dws[5], acc[5], t[5];
    if (MODE == SW_FWD || MODE == SW_TOP) {
#pragma unroll
        for (int k = 0; k < 5; k++) acc[k] = T(P.M[k * N + c]);
        // lower neighbours of the cell's block; with two block passes, the
        // second also takes every neighbour in another block, with the first
        // pass's increment
        auto lower = [&](const Entries &E, int b) {
#pragma unroll
            for (int k = 0; k < MAXV; k++) {
                const int j = E.nbr[k], fl = E.flag[k];
                if (!(fl & CF_VALID) || j < 0) continue;
                const bool cross = (fl & CF_OTHER) && P.dWx;
                if (!(fl & CF_LOWER) && !cross) continue;
                sweep_term<T, ROE>(P, ip, W, w, E.face[k], MAXV * b + k, j, dws, cfl, 0, t, cross ? P.dWx : P.dW,
                                   cross);
#pragma unroll
                for (int m = 0; m < 4; m++) acc[m] = acc_sub(acc[m], t[m]);
                acc[4] = acc_add(acc[4], t[4]);
            }
        };
        lower(E0, c);
        if (ovf >= 0) lower(entries(P, ovf), ovf);
        if (ROE) {
            dinv_apply(P, c, acc, dws);
        } else {
            const T iD = T(1) / D;
#pragma unroll
            for (int k = 0; k < 4; k++) dws[k] = acc[k] * iD;
        }
        dws[4] = ip.sa ? acc[4] / (odt + T(P.sadiag[c])) : T(0);
        if (MODE == SW_FWD) {
#pragma unroll
            for (int k = 0; k < 5; k++) P.dW[k * N + c] = dws[k];
            return 0.0;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 5; k++) dws[k] = P.dW[k * N + c];
    }
#pragma unroll
    for (int k = 0; k < 5; k++) acc[k] = T(0);
    auto upper = [&](const Entries &E, int b) {
#pragma unroll
        for (int k = 0; k < MAXV; k++) {
            const int j = E.nbr[k], fl = E.flag[k];
            if (!(fl & CF_VALID) || (j >= 0 && (fl & (CF_LOWER | CF_OTHER)))) continue;
            sweep_term<T, ROE>(P, ip, W, w, E.face[k], MAXV * b + k, j, dws, cfl, 0, t, P.dW);
#pragma unroll
            for (int m = 0; m < 5; m++) acc[m] = acc_add(acc[m], t[m]);
        }
    };
    upper(E0, c);
    if (ovf >= 0) upper(entries(P, ovf), ovf);
    T d[5];
    if (ROE) {
        T y[4];
        dinv_apply(P, c, acc, y);
#pragma unroll
        for (int k = 0; k < 4; k++) d[k] = dws[k] - y[k];
    } else {
        const T iD = T(1) / D;
#pragma unroll
        for (int k = 0; k < 4; k++) d[k] = dws[k] - acc[k] * iD;
    }
    d[4] = ip.sa ? dws[4] + acc[4] / (odt + T(P.sadiag[c])) : T(0);
#pragma unroll
    for (int k = 0; k < 5; k++) P.dW[k * N + c] = d[k];
    if (MODE == SW_BWD_ONLY) return 0.0;
    double dd[5];
#pragma unroll
    for (int k = 0; k < 5; k++) dd[k] = double(d[k]);
    return apply_update(P, c, inst, w, dd);
}

// sweep_cell on a quad of lanes (q = 0..3, one cell per aligned quad): lane
// q takes entry q of each of the cell's entry blocks, so a cell's neighbour
// terms are formed side by side instead of one after another, and the
// terms are combined on every lane of the quad in entry order (quad_fold),
// which gives the same numbers as sweep_cell.  Lane 0 stores and returns
// the Eq.40 ratio; the other lanes return 0.  Cells below lev1 (the first
// wavefront) have no stored forward increment: their own and their
// neighbours' are formed by first_front_incr.
template <typename T, int MODE, bool ONE, bool ROE>
__device__ __forceinline__ double sweep_quad(const Params<T> &P, int c, int q, int lev1, int &inst)
{
    const int N = P.nc;
    inst = live_inst<ONE>(P, P.cinst, c);   // the same on the four lanes
    if (inst < 0) return 0.0;
    const InstScalars &sc = P.is[inst];
    const InstParam &ip = P.ip[inst];
    const double *W = cur_state(P, inst);
    const T cfl = T(sc.cfl);
    double w[5];
#pragma unroll
    for (int k = 0; k < 5; k++) w[k] = W[k * N + c];
    const int f0 = P.cf_face[MAXV * c + q], j0 = P.cf_nbr[MAXV * c + q], fl0 = P.cf_flag[MAXV * c + q];
    const int nxt = quad_get<3>(fl0) >> CF_NEXT_SHIFT;
    const int ovf = nxt ? N + nxt - 1 : -1;   // a polygon's overflow block, or -1
    const T odt = T(P.lamc[c]) / cfl;
    const T D = odt + T(P.lsum[c]);
    T dws[5], acc[5], t[5];
    if (MODE == SW_FWD || MODE == SW_TOP) {
#pragma unroll
        for (int k = 0; k < 5; k++) acc[k] = T(P.M[k * N + c]);
        // lower neighbours of the cell's block; with two block passes, the
        // second also takes every neighbour in another block, with the first
        // pass's increment
        auto lower = [&](int f, int e, int j, int fl) {
#pragma unroll
            for (int m = 0; m < 5; m++) t[m] = T(0);
            const bool cross = (fl & CF_OTHER) && P.dWx;
            if ((fl & CF_VALID) && j >= 0 && ((fl & CF_LOWER) || cross))
                sweep_term<T, ROE>(P, ip, W, w, f, e, j, dws, cfl, cross ? 0 : lev1, t, cross ? P.dWx : P.dW, cross);
#pragma unroll
            for (int m = 0; m < 4; m++) acc[m] = quad_fold<true>(acc[m], t[m]);
            acc[4] = quad_fold<false>(acc[4], t[4]);
        };
        lower(f0, MAXV * c + q, j0, fl0);
        if (ovf >= 0)
            lower(P.cf_face[MAXV * ovf + q], MAXV * ovf + q, P.cf_nbr[MAXV * ovf + q], P.cf_flag[MAXV * ovf + q]);
        if (ROE) {
            dinv_apply(P, c, acc, dws);
        } else {
            const T iD = T(1) / D;
#pragma unroll
            for (int k = 0; k < 4; k++) dws[k] = acc[k] * iD;
        }
        dws[4] = ip.sa ? acc[4] / (odt + T(P.sadiag[c])) : T(0);
        if (MODE == SW_FWD) {
            if (q == 0) {
#pragma unroll
                for (int k = 0; k < 5; k++) P.dW[k * N + c] = dws[k];
            }
            return 0.0;
        }
    } else if (c < lev1) {
        first_front_incr<T, ROE>(P, ip, c, cfl, dws);
    } else {
#pragma unroll
        for (int k = 0; k < 5; k++) dws[k] = P.dW[k * N + c];
    }
#pragma unroll
    for (int k = 0; k < 5; k++) acc[k] = T(0);
    auto upper = [&](int f, int e, int j, int fl) {
#pragma unroll
        for (int m = 0; m < 5; m++) t[m] = T(0);
        if ((fl & CF_VALID) && !(j >= 0 && (fl & (CF_LOWER | CF_OTHER))))
            sweep_term<T, ROE>(P, ip, W, w, f, e, j, dws, cfl, lev1, t, P.dW);
#pragma unroll
        for (int m = 0; m < 5; m++) acc[m] = quad_fold<false>(acc[m], t[m]);
    };
    upper(f0, MAXV * c + q, j0, fl0);
    if (ovf >= 0)
        upper(P.cf_face[MAXV * ovf + q], MAXV * ovf + q, P.cf_nbr[MAXV * ovf + q], P.cf_flag[MAXV * ovf + q]);
    if (q != 0) return 0.0;
    T d[5];
    if (ROE) {
        T y[4];
        dinv_apply(P, c, acc, y);
#pragma unroll
        for (int k = 0; k < 4; k++) d[k] = dws[k] - y[k];
    } else {
        const T iD = T(1) / D;
#pragma unroll
        for (int k = 0; k < 4; k++) d[k] = dws[k] - acc[k] * iD;
    }
    d[4] = ip.sa ? dws[4] + acc[4] / (odt + T(P.sadiag[c])) : T(0);
#pragma unroll
    for (int k = 0; k < 5; k++) P.dW[k * N + c] = d[k];
    if (MODE == SW_BWD_ONLY) return 0.0;
    double dd[5];
#pragma unroll
    for (int k = 0; k < 5; k++) dd[k] = double(d[k]);
    return apply_update(P, c, inst, w, dd);
}

// One wave per instance (block i): the L2 norms from the partial sums (in
// a fixed order), the drop reference and limiter freezing, then accept
// (flip the state buffer) or reject and freeze the instance, the Eq.40
// maximum, slots reset for the next iteration.
template <typename T>
__global__ __launch_bounds__(64) void k_commit(Params<T> P, int it)
{
    const int i = blockIdx.x, lane = threadIdx.x;
    InstScalars *s = &P.is[i];
    if (s->halt) return;
    double e40 = wave_max(slot_lane(P.slot, i, SL_E40));
    double x = 0.0, y = 0.0;
    // unrolled so that the loads of several slices are in flight together
    // (the sums keep their order)
#pragma unroll 8
    for (int k = lane; k < P.rb; k += warpSize) {
        x += P.ipart[2 * (i * P.rb + k)];
        y += P.ipart[2 * (i * P.rb + k) + 1];
    }
    x = wave_sum(x);
    y = wave_sum(y);
    int bad = s->bad;
    *slot_at(P.slot, i, SL_DTMIN, lane) = 0x7ff0000000000000ull;
    *slot_at(P.slot, i, SL_E40, lane) = 0ull;
    if (lane != 0) return;
    const double l2 = sqrt(x), sal2 = sqrt(y);
    // the drop is measured from the largest ||M_rho||_2 so far
    if (s->ncommit == 0 || l2 > s->res0) s->res0 = l2;
    // limiter freezing: from the next iteration on, the factors just computed
    if (P.limiter && P.limiter_freeze > 0.0 && !s->phi_frozen && l2 <= P.limiter_freeze * s->res0) s->phi_frozen = 1;
    s->res_l2 = l2;
    s->sa_l2 = sal2;
    s->e40 = e40;
    if (it < P.hist_cap) {
        double *e = P.hist + (size_t)HIST_W * ((size_t)it * P.ninst + i);
        e[0] = l2; e[4] = e40; e[5] = sal2;
    }
    if (bad) s->halt = 1;
    else s->ncommit += 1;
}

// One wavefront of cells [c0, c1), four lanes per cell (sweep_quad)
template <typename T, int MODE, bool ONE, bool ROE>
__global__ __launch_bounds__(256) void k_sweep(Params<T> P, int c0, int c1, int lev1)
{
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    const int c = c0 + (t >> 2);
    int inst = -1;
    double e = 0.0;
    if (c < c1) e = sweep_quad<T, MODE, ONE, ROE>(P, c, t & 3, lev1, inst);
    if (MODE != SW_FWD) slot_update<false>(P.slot, SL_E40, inst, e);
}

// The whole sweep in one workgroup: wavefront after wavefront, separated by
// workgroup barriers (all waves of a workgroup share one CU and its L1, so
// the barrier orders the dW writes of one wavefront before the reads of the
// next).  Used when wavefronts are many and narrow: the time per wavefront
// is latency, so the backward sweep leaves the update (Eq.17, Eq.40) to one
// parallel pass afterwards (k_update) instead of adding its loads and stores
// to every step.
// ONE (a context of one instance) makes the instance index a constant, so
// its scalars come through scalar loads instead of a dependent vector load
// chain on every wavefront.
template <typename T, bool FWD, bool ONE, bool ROE>
__global__ __launch_bounds__(512) void k_sweep_wg(Params<T> P, const int *lev_off, int nlev)
{
    for (int i = 0; i < nlev; i++) {
        int l = FWD ? i : nlev - 1 - i;
        int c0 = lev_off[l], c1 = lev_off[l + 1];
        for (int c = c0 + (int)threadIdx.x; c < c1; c += (int)blockDim.x) {
            int inst;
            (void)sweep_cell<T, FWD ? SW_FWD : SW_BWD_ONLY, ONE, ROE>(P, c, inst);
        }
        __syncthreads();
    }
}

// The whole sweep of one sweep block per wave: the block's wavefronts one
// after another, each cell of a wavefront on a quad of lanes (lane q forms
// the term of entry q, sweep_quad; 16 cells per step, and a block's
// wavefront holds a few cells).  Blocks do not couple in the sweeps, so no
// wave waits for another; inside the one-wave workgroup the barrier after
// each wavefront orders its dW writes before the next wavefront's reads.
// As in the one-workgroup sweep, the backward pass leaves the update to
// k_update.
template <typename T, bool FWD, bool ONE, bool ROE>
__global__ __launch_bounds__(64) void k_sweep_blk(Params<T> P, const int *bl_off, const int *bl_lo, const int *bl_hi)
{
    const int gb = blockIdx.x;
    const int k0 = bl_off[gb], k1 = bl_off[gb + 1];
    const int q = (int)threadIdx.x & 3, cell = (int)threadIdx.x >> 2;
    for (int i = 0; i < k1 - k0; i++) {
        const int k = FWD ? k0 + i : k1 - 1 - i;
        const int c0 = bl_lo[k], c1 = bl_hi[k];
        for (int c = c0 + cell; c < c1; c += 16) {   // the four lanes of a quad take the same cell
            int inst;
            (void)sweep_quad<T, FWD ? SW_FWD : SW_BWD_ONLY, ONE, ROE>(P, c, q, 0, inst);
        }
        __syncthreads();
    }
}

// W^{n+1} = W^n + dW for every cell from the finished backward sweep (the
// same arithmetic as the fused update of the per-wavefront path)
template <typename T, bool ONE>
__global__ __launch_bounds__(256) void k_update(Params<T> P)
{
    const int N = P.nc;
    int c = xcd_block() * blockDim.x + threadIdx.x;
    int inst = -1;
    double e = 0.0;
    if (c < N) {
        inst = live_inst<ONE>(P, P.cinst, c);
        if (inst >= 0) {
            const double *W = cur_state(P, inst);
            double w[5], d[5];
#pragma unroll
            for (int k = 0; k < 5; k++) {
                w[k] = W[k * N + c];
                d[k] = double(P.dW[k * N + c]);
            }
            e = apply_update(P, c, inst, w, d);
        }
    }
    slot_update<false>(P.slot, SL_E40, inst, e);
}

// exact distance from each centroid to the nearest wall segment of its instance
__global__ __launch_bounds__(256) void k_wall_distance(int nc, const double *xc, const double *yc, const int *cinst,
                                                       const int *woff, const double *seg, double *d)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int i = cinst[c];
    double px = xc[c], py = yc[c], best = 1e300;
    for (int s = woff[i]; s < woff[i + 1]; s++) {
        double ax = seg[4 * s], ay = seg[4 * s + 1], bx = seg[4 * s + 2], by = seg[4 * s + 3];
        double ex = bx - ax, ey = by - ay;
        double t = ((px - ax) * ex + (py - ay) * ey) / (ex * ex + ey * ey);
        t = fmin(fmax(t, 0.0), 1.0);
        double dx = px - ax - t * ex, dy = py - ay - t * ey;
        best = fmin(best, sqrt(dx * dx + dy * dy));
    }
    d[c] = best;
}

__global__ void k_gather_faces(int n, const int *faces, const double *frec, int nf, double *out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int f = faces[i];
    const double *r = frec + FR_STRIDE * (size_t)f;
    out[4 * i] = r[FR_F0];
    out[4 * i + 1] = r[FR_F1];
    out[4 * i + 2] = r[FR_F2];
    out[4 * i + 3] = r[FR_F3];
}

__global__ void k_fill_instance(int n, const int *cells, int nc, double w0, double w1, double w2, double w3,
                                double w4, double *W)
{
    int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int c = cells[u];
    W[c] = w0; W[nc + c] = w1; W[2 * nc + c] = w2; W[3 * nc + c] = w3; W[4 * nc + c] = w4;
}

// to_instance: dst (5 x nc, internal order) <- src (5 x n, upload order);
// else the reverse
__global__ void k_copy_instance(int n, const int *cells, int nc, const double *src, double *dst, int to_instance)
{
    int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int c = cells[u];
#pragma unroll
    for (int k = 0; k < 5; k++) {
        if (to_instance) dst[(size_t)k * nc + c] = src[(size_t)k * n + u];
        else dst[(size_t)k * n + u] = src[(size_t)k * nc + c];
    }
}

// ---------------------------------------------------------------- launchers

static inline int nblk(int n, int b) { return (n + b - 1) / b; }

template <typename T> void launch_reset(const Launch &L, const Params<T> &P, int mode, int inst)
{
    hipLaunchKernelGGL(k_reset<T>, dim3(1), dim3(64), 0, L.s, P, mode, inst);
}
// ONE-instance variants of the cell and face kernels for contexts of one
// instance (see live_inst)
#define LAUNCH_ONE(K, T, grid, block, ...)                                            \
    do {                                                                              \
        if (P.ninst == 1) hipLaunchKernelGGL((K<T, true>), grid, block, 0, L.s, __VA_ARGS__); \
        else hipLaunchKernelGGL((K<T, false>), grid, block, 0, L.s, __VA_ARGS__);     \
    } while (0)

template <typename T> void launch_prep(const Launch &L, const Params<T> &P)
{
    LAUNCH_ONE(k_prep, T, dim3(nblk(P.nc, L.block[0])), dim3(L.block[0]), P);
}
template <typename T> void launch_explicit(const Launch &L, const Params<T> &P)
{
    LAUNCH_ONE(k_explicit, T, dim3(nblk(P.nc, L.block[0])), dim3(L.block[0]), P);
}
template <typename T> void launch_commit(const Launch &L, const Params<T> &P, int it)
{
    hipLaunchKernelGGL(k_commit<T>, dim3(P.ninst), dim3(64), 0, L.s, P, it);
}
template <typename T> void launch_flux(const Launch &L, const Params<T> &P)
{
    if (L.flux_pair) LAUNCH_ONE(k_flux2, T, dim3(nblk(2 * P.nf, L.block[1])), dim3(L.block[1]), P);
    else LAUNCH_ONE(k_flux, T, dim3(nblk(P.nf, L.block[1])), dim3(L.block[1]), P);
}
template <typename T> void launch_gather(const Launch &L, const Params<T> &P)
{
    LAUNCH_ONE(k_gather, T, dim3(nblk(P.nc, L.block[2])), dim3(L.block[2]), P);
}
template <typename T> void launch_reduce(const Launch &L, const Params<T> &P, int it)
{
    hipLaunchKernelGGL(k_reduce<T>, dim3(P.ninst * (P.rb + 1)), dim3(256), 0, L.s, P, it);
}
// the sweep kernels K<T, X, ONE, ROE> come in four variants: one instance or
// several (ONE), the scalar or the Roe-matrix operator (ROE)
#define LAUNCH_SWEEP(K, X, grid, block, ...)                                                         \
    do {                                                                                             \
        const bool one_ = P.ninst == 1, roe_ = P.dinv != nullptr;                                    \
        if (one_ && !roe_) hipLaunchKernelGGL((K<T, X, true, false>), grid, block, 0, L.s, __VA_ARGS__); \
        else if (!roe_) hipLaunchKernelGGL((K<T, X, false, false>), grid, block, 0, L.s, __VA_ARGS__);   \
        else if (one_) hipLaunchKernelGGL((K<T, X, true, true>), grid, block, 0, L.s, __VA_ARGS__);      \
        else hipLaunchKernelGGL((K<T, X, false, true>), grid, block, 0, L.s, __VA_ARGS__);               \
    } while (0)

template <typename T> void launch_sweep(const Launch &L, const Params<T> &P, int c0, int c1, int mode, int lev1)
{
    if (c1 <= c0) return;
    dim3 g(nblk(4 * (c1 - c0), L.block[3])), b(L.block[3]);
    if (mode == SW_FWD) LAUNCH_SWEEP(k_sweep, SW_FWD, g, b, P, c0, c1, lev1);
    else if (mode == SW_BWD) LAUNCH_SWEEP(k_sweep, SW_BWD, g, b, P, c0, c1, lev1);
    else LAUNCH_SWEEP(k_sweep, SW_TOP, g, b, P, c0, c1, lev1);
}
template <typename T> void launch_sweep_wg(const Launch &L, const Params<T> &P, const int *lev_off, int nlev, bool fwd)
{
    if (fwd) {
        LAUNCH_SWEEP(k_sweep_wg, true, dim3(1), dim3(512), P, lev_off, nlev);
    } else {
        LAUNCH_SWEEP(k_sweep_wg, false, dim3(1), dim3(512), P, lev_off, nlev);
        LAUNCH_ONE(k_update, T, dim3(nblk(P.nc, L.block[3])), dim3(L.block[3]), P);
    }
}
template <typename T>
void launch_sweep_blk(const Launch &L, const Params<T> &P, const int *bl_off, const int *bl_lo, const int *bl_hi,
                      int ngb, bool fwd, bool update)
{
    if (ngb <= 0) return;
    if (fwd) {
        LAUNCH_SWEEP(k_sweep_blk, true, dim3(ngb), dim3(64), P, bl_off, bl_lo, bl_hi);
    } else {
        LAUNCH_SWEEP(k_sweep_blk, false, dim3(ngb), dim3(64), P, bl_off, bl_lo, bl_hi);
        if (update) LAUNCH_ONE(k_update, T, dim3(nblk(P.nc, L.block[3])), dim3(L.block[3]), P);
    }
}
template <typename T> void launch_roe_diag(const Launch &L, const Params<T> &P)
{
    LAUNCH_ONE(k_roe_diag, T, dim3(nblk(P.nc, L.block[2])), dim3(L.block[2]), P);
}
void launch_wall_distance(const Launch &L, int nc, const double *xc, const double *yc, const int *cinst,
                          const int *woff, const double *wseg, double *dwall)
{
    hipLaunchKernelGGL(k_wall_distance, dim3(nblk(nc, 256)), dim3(256), 0, L.s, nc, xc, yc, cinst, woff, wseg, dwall);
}
void launch_gather_faces(const Launch &L, int n, const int *faces, const double *frec, int nf, double *out)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_faces, dim3(nblk(n, 256)), dim3(256), 0, L.s, n, faces, frec, nf, out);
}
void launch_fill_instance(const Launch &L, int n, const int *cells, int nc, const double *Winf, double *W)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_instance, dim3(nblk(n, 256)), dim3(256), 0, L.s, n, cells, nc, Winf[0], Winf[1],
                       Winf[2], Winf[3], Winf[4], W);
}
void launch_copy_instance(const Launch &L, int n, const int *cells, int nc, const double *src, double *dst,
                          bool to_instance)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy_instance, dim3(nblk(n, 256)), dim3(256), 0, L.s, n, cells, nc, src, dst,
                       to_instance ? 1 : 0);
}

#define INST(T)                                                                                    \
    template void launch_reset<T>(const Launch &, const Params<T> &, int, int);                    \
    template void launch_prep<T>(const Launch &, const Params<T> &);                               \
    template void launch_flux<T>(const Launch &, const Params<T> &);                               \
    template void launch_gather<T>(const Launch &, const Params<T> &);                             \
    template void launch_reduce<T>(const Launch &, const Params<T> &, int);                        \
    template void launch_roe_diag<T>(const Launch &, const Params<T> &);                           \
    template void launch_sweep<T>(const Launch &, const Params<T> &, int, int, int, int);          \
    template void launch_commit<T>(const Launch &, const Params<T> &, int);                        \
    template void launch_explicit<T>(const Launch &, const Params<T> &);                           \
    template void launch_sweep_wg<T>(const Launch &, const Params<T> &, const int *, int, bool);                 \
    template void launch_sweep_blk<T>(const Launch &, const Params<T> &, const int *, const int *, const int *,  \
                                      int, bool, bool);
INST(double)
INST(float)

}  // namespace igks

// igks_dev.h - data shared by the host driver and the HIP kernels of
// libigks (gfx950).  Internal to the library.
//
// A context holds one or more independent instances (mesh + flow
// condition).  Their cells and faces are concatenated; every kernel handles
// all instances in one launch and reads the per-instance free stream and
// scalars through the cell's (or face's) instance index.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace igks {

// Sec. 2.1 after Eq.2: K = 3 internal degrees of freedom; gamma = (K+4)/(K+2).
constexpr int KDOF = 3;
constexpr double GAMMA = (KDOF + 4.0) / (KDOF + 2.0);

enum { BC_FREESTREAM = 1, BC_SYMMETRY = 2, BC_WALL = 3, BC_OUTFLOW = 4, BC_FARFIELD = 5, BC_MOVING_WALL = 6 };

// cell -> face entry flags
constexpr int CF_OWNER = 1;   // the cell is the face's owner (normal points outward)
constexpr int CF_LOWER = 2;   // interior neighbour of the same sweep block with a smaller upload index
constexpr int CF_VALID = 4;   // the entry exists (triangles leave their fourth entry empty)
constexpr int CF_OTHER = 16;  // interior neighbour in another sweep block (left out of the sweeps)
// A polygon's faces and vertices beyond the fourth sit in an overflow block
// of four more (block nc + o); the last entry of a block carries o + 1 in
// the flag bits from CF_NEXT_SHIFT on (0: no further block).
constexpr int CF_NEXT_SHIFT = 8;

constexpr int MAXV = 4;       // entries and vertices per block (triangles pad by repeating a vertex)
constexpr int MAXP = 8;       // vertices of the largest cell (two blocks)
constexpr int HIST_W = 6;     // doubles per history entry
// Atomic min / max targets: NSLOT slots per instance and quantity, each on
// a 128-byte line of its own (atomics on one line are carried out one after
// another), holding non-negative doubles as integers (they compare like
// their bit patterns, so min / max of them is exact and order independent).
constexpr int NSLOT = 64;
constexpr int SLOT_STRIDE = 16;   // unsigned long longs from one slot to the next
enum { SL_DTMIN = 0, SL_RESINF = 1, SL_E40 = 2, NSL = 3 };   // Eq.23 minimum, max |M|, Eq.40 maximum
constexpr int NORM_SLICE = 1024;   // squares per block of the residual-norm partial sums
// face record layout (Params::frec)
constexpr int FR_STRIDE = 8, FR_F0 = 0, FR_F1 = 1, FR_LAM = 2, FR_SAF = 3, FR_F2 = 4, FR_F3 = 5, FR_SAG = 6, FR_SAK = 7;
constexpr int NCLASS = 4;     // kernel classes with a tunable block size: prep, flux, gather, sweep

// Free stream of one instance (read-only while iterating).
struct InstParam {
    double Winf[5];
    double lam_inf, mu_inf, p_inf;
    double tw;                 // RT of isothermal walls; 0: adiabatic walls
    int sa;
    int pad;
};

// Scalars of one instance, updated on the device.
struct InstScalars {
    double dt;                              // Eq.23 time step of the current iteration
    double cfl;                             // implicit CFL of the current iteration
    double res_inf_prev;                    // ||M||_inf of the previous iteration
    double res0;                            // ||M_rho||_2 of iteration 0
    double res_l2, sa_l2, res_inf, e40;
    int ncommit;                            // committed iterations; its parity picks the state buffer
    int bad;                                // the last update produced a non-physical state
    int halt;                               // the instance is frozen (rejected update)
    int phi_frozen;                         // limiter factors held (limiter_freeze)
};

template <typename T>
struct Params {
    int nc, nf, ninst;
    int limiter, visc_sr, mu_law, cfl_mode;
    double cfl_init, cfl_min, cfl_max, cfl_flux;
    double limiter_freeze;     // drop at which an instance's limiter factors are held; 0 never
    int tau_jump;              // add dt |p_l - p_r| / (p_l + p_r) to the collision time
    double *phi;               // 4 x nc: the last computed limiter factors
    const int *cinst, *finst;  // instance of each cell / face
    const InstParam *ip;
    InstScalars *is;
    unsigned long long *slot;  // ninst x NSL x NSLOT slots, SLOT_STRIDE apart
    // cell arrays (SoA, internal order)
    double *Wa, *Wb;           // state ping-pong, 5 x nc
    double *grad;              // limited gradients: d/dx of rho, rhoU, rhoV, rhoE, then d/dy
    double *lamc;              // Eq.21 spectral radius sum
    double *vort;              // |dV/dx - dU/dy| (unlimited gradients)
    double *nu;                // laminar kinematic viscosity
    double *M;                 // residual: 4 flow components + SA right-hand side
    double *lsum;              // 1/2 sum lambda S (Eq.20 diagonal)
    double *sadiag;            // SA diagonal without Omega/dt
    double *r2;                // squares for the norms, M_rho^2 then R_SA^2, at the cell's ipos
    T *dW;                     // LU-SGS increment, 5 x nc
    const T *dWx;              // a first block pass's increments, whose cross-block terms the
                               // forward sweep takes (two block passes); null otherwise
    T *dinv;                   // Roe-matrix operator: the inverse of each cell's 4x4 LU-SGS
                               // diagonal block, entry (r, k) at (4 r + k) nc + c; null with
                               // the scalar operator
    int roe_kin;               // Roe-matrix operator with the kinetic wave magnitudes
    const double *xc, *yc, *area, *lsinv, *dwall;
    const double *vtx;         // vertex offsets from the centroid: (x, y) of slot v of block b at (2v) nb + b
    int nb;                    // entry / vertex blocks: nc + overflow blocks
    // cell-face entries, MAXV per block (entry MAXV b + k; block b = c, then
    // the overflow block of a polygon): face, neighbour (-1: ghost cell),
    // flags, centroid offsets to the neighbour (or ghost)
    const int *cf_face, *cf_nbr, *cf_flag;
    const double *cf_dx, *cf_dy;
    // per entry, the face seen from the entry's cell: the normal pointing out
    // of the cell and the face length (a cell's entries are contiguous)
    const double *enx, *eny, *es;
    // face arrays (internal face order)
    const int *fl, *fr, *fbc;
    // fidl, fidr, firn: 1/d_l, 1/d_r (centroid-face normal distances; d_r = d_l
    // on a boundary face) and 1/|r.n| (centroid to centroid, 2 d_l on a boundary)
    const double *fnx, *fny, *flen, *frl, *frr, *fidl, *fidr, *firn;
    // nf x FR_STRIDE face records, one 64-byte record per face, so that a
    // cell reading a face's outputs through its entries touches one cache
    // line: FR_F0, FR_F1, FR_F2, FR_F3 the time-averaged flux times length
    // (global frame), FR_LAM the spectral radius, FR_SAF the SA
    // (-F_inv + F_vis) S, FR_SAG (nu~_r - nu~_l)/|r.n| S, FR_SAK the SA
    // diffusion coefficient of the face times S/|r.n|.  Each half of a record
    // is written by one 16-byte store per pair of values.
    double *frec;
    // the spectral radius and the SA diffusion coefficient again, packed
    // one value per face: the sweeps read only these two, and a packed
    // array puts sixteen faces in a cache line where the records put two
    double *flam, *fsak;
    // per-instance cell lists (internal ids, ascending) for the norms
    const int *icell, *ioff;
    const int *ipos;           // position of each cell in icell
    // processing order of the cell kernels k_prep and k_gather: cells grouped
    // in spatial tiles, each tile's wavefronts one after another, so that a
    // cell and its neighbours (which lie in other wavefronts) are read by the
    // same XCD close together in time
    const int *cperm;
    double *ipart;             // ninst x rb x 2 partial sums
    int rb;                    // partial sums per instance: slices of NORM_SLICE squares
    double *hist;              // HIST_W x ninst x hist_cap
    int hist_cap;
};

// launchers (igks_kernels.hip)
struct Launch {
    hipStream_t s;
    int block[NCLASS];        // prep, flux, gather, sweep
    bool flux_pair;           // flux on two lanes per face (else one)
};
template <typename T> void launch_reset(const Launch &L, const Params<T> &P, int mode, int inst);
template <typename T> void launch_prep(const Launch &L, const Params<T> &P);
template <typename T> void launch_flux(const Launch &L, const Params<T> &P);
template <typename T> void launch_gather(const Launch &L, const Params<T> &P);
// it: the iteration's index in the current chunk (its history entry)
template <typename T> void launch_reduce(const Launch &L, const Params<T> &P, int it);
template <typename T> void launch_roe_diag(const Launch &L, const Params<T> &P);
// one wavefront of cells [c0, c1) of the sweeps; mode 0 forward, 1 backward,
// 2 both (the last wavefront).  Backward steps also update the state
// (Eq.17); launch_commit then accepts or rejects the iteration of every
// instance.  Cells below lev1 form the first wavefront, whose forward step
// is not launched (its increments are formed where they are read); 0: every
// forward increment is stored.
template <typename T> void launch_sweep(const Launch &L, const Params<T> &P, int c0, int c1, int mode, int lev1);
template <typename T> void launch_sweep_wg(const Launch &L, const Params<T> &P, const int *lev_off, int nlev, bool fwd);
// the whole sweep, one wave per sweep block (ngb blocks; block gb's k-th
// wavefront = cells [bl_lo[bl_off[gb] + k], bl_hi[bl_off[gb] + k])); the
// backward sweep is followed by the update of every cell unless `update` is
// false (the first of two block passes)
template <typename T>
void launch_sweep_blk(const Launch &L, const Params<T> &P, const int *bl_off, const int *bl_lo, const int *bl_hi,
                      int ngb, bool fwd, bool update = true);
template <typename T> void launch_commit(const Launch &L, const Params<T> &P, int it);
// explicit step (Eq.15, local time steps) in place of the sweeps
template <typename T> void launch_explicit(const Launch &L, const Params<T> &P);
void launch_wall_distance(const Launch &L, int nc, const double *xc, const double *yc, const int *cinst,
                          const int *woff, const double *wseg, double *dwall);
void launch_gather_faces(const Launch &L, int n, const int *faces, const double *frec, int nf, double *out);
void launch_fill_instance(const Launch &L, int n, const int *cells, int nc, const double *Winf, double *W);
void launch_copy_instance(const Launch &L, int n, const int *cells, int nc, const double *src, double *dst,
                          bool to_instance);

}  // namespace igks

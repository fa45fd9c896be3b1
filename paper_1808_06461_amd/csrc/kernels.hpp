// Kernel argument blocks and launcher declarations (internal to the library).
#pragma once
#include "common.hpp"

namespace chn {

struct PlaneDims {
  int n1h, n2, n3, p1, p3;
  double lx, lz;
};

template <typename T> struct ZinvArgs {
  const c2<T>* in[6];  // u1, u2, u3, omega1, omega2, omega3 spectral [n2][n1h][n3];
                       // in[4] == nullptr: omega2 = i b u1 - i a u3 formed here
  c2<T>* out;          // [n2][nslot][p3][n1h]
  const c2<T>* tw;     // twiddles of the p3 plan
  FftPlan plan;
  PlaneDims d;
  int K;               // kx lines per workgroup
  int lstride;         // LDS line stride (complex elements)
  int nfields;         // 6: u1 u2 u3 omega1 omega2 omega3; 3: u1 u2 u3
  int nslot;           // field slots per plane in `out`
  int zero_mean;       // nonzero: the (0,0) coefficient of every input is taken as 0
  int y0, ny;          // planes y0 .. y0 + ny - 1 of the inputs; `out` holds them from plane 0
  int fixed;           // nonzero: compile-time radix schedule where one exists for the plan
  unsigned* guard;     // instability guard (common.hpp) whose CFL word the launch
                       // with y0 == 0 resets; nullptr outside the time step
  int pipe;            // nonzero: the next field's loads overlap this field's transform
                       // (256-thread launches whose field fits the staging registers)
  unsigned in_f32;     // bit f set: in[f] points to float32 coefficients, widened on
                       // load (float64 transforms of float32 data; 0 for float32 transforms)
};

template <typename T> struct XpassArgs {
  c2<T>* buf;          // [n2][6][p3][n1h], transformed in place
  const c2<T>* tw;     // twiddles of the p1 plan
  FftPlan plan;
  PlaneDims d;
  int lstride;
  double* rowsum;      // [2][n2][p3] sums over x of H1 and H3
  double* rowcfl;      // [n2][p3] max over x of |u1|/dx + |u2|/dy + |u3|/dz
  double inv_dx, inv_dz;
  const double* inv_dy;  // [n2]
  int rows;              // rows per workgroup: 2, 4, 8 (3 rows lines in LDS) or 1 (long rows)
  int y0, ny;            // buf holds planes y0 .. y0 + ny - 1 (from its plane 0)
  int fixed;             // nonzero: compile-time radix schedule where one exists for the plan
  unsigned* guard;       // instability guard: every workgroup raises word 0 to its
                         // CFL maximum (nullptr outside the time step)
};

template <typename T, typename TO> struct ZfwdArgs {
  const c2<T>* buf;    // [n2][6][p3][n1h]
  c2<TO>* out[3];      // H1, H2, H3 spectral [n2][n1h][n3]
  const c2<T>* tw;
  FftPlan plan;
  PlaneDims d;
  int K;
  int lstride;
  double scale;        // 1 / (p1 p3)
  int y0, ny;          // buf holds planes y0 .. y0 + ny - 1 (from its plane 0); out is global
  int fixed;           // nonzero: compile-time radix schedule where one exists for the plan
  int pipe;            // nonzero: the next field's loads overlap this field's transform
};

template <typename T> hipError_t launch_zinv(const ZinvArgs<T>& a, hipStream_t st);
template <typename T> hipError_t launch_xpass(const XpassArgs<T>& a, hipStream_t st);
// x-pass kernel choice for rows of p1 points of bytes_per_value-byte complex values
bool xpass_two_rows(int p1, int bytes_per_value);
int xrow_threads(int p1, int bytes_per_value);  // 0: too long
// Staging checks of the transforms: whether nlines lines of the plan over nt
// threads fit m staged values per thread in every pass; the staging a z pass
// of K lines would use (0: none fits); whether the long-row x pass fits.
bool staging_fits(const FftPlan& pl, int nlines, int nt, int m);
int z_staging(const FftPlan& pl, int K, int bytes_per_value);
bool xrow_fits(const FftPlan& pl, int bytes_per_value);
template <typename T, typename TO> hipError_t launch_zfwd(const ZfwdArgs<T, TO>& a, hipStream_t st);

// ---------------------------------------------------------------- filter stage
// The products are formed on an f1 x f3 grid with f > 2 h + kc (h = highest
// stored wavenumber of the direction, kc the cut-off): every product mode
// that aliases onto a retained one lies beyond 2 h, so the retained modes are
// exact on that grid (the 3/2 grid of the time step is one such grid).
template <typename T> struct XfilterArgs {
  const c2<T>* buf;      // [n2][3][f3][n1h]: the three fields after the z inverse (float64 in use)
  double2* out;          // per plane y at out + y * plane_stride: [6][f3][kcx+1] (trace: [1][f3][kcx+1])
  size_t plane_stride;   // in double2 elements
  const c2<T>* tw;       // f1 plan twiddles, phase precision (inverse)
  FftPlan plan;
  const double2* tw_d;   // f1 plan twiddles, float64 (forward)
  int n1h, n2, f1, f3;
  int lst, lsd;          // LDS line strides (phase-precision and float64 lines)
  int kcx;
  int trace;             // nonzero: one product, the sum of the three squares
};

// The three fields' coefficients, spectral [n2][n1h][n3]: complex float64, or
// complex float32 where bit i of `f32` is set.
struct FieldsIn {
  const void* u[3];
  unsigned f32;
};

struct ZfilterArgs {
  const double2* xout;   // output of k_xfilter
  size_t plane_stride;
  FieldsIn u;            // the three fields (full mode set)
  double2* pp;           // [6][n2][kcx+1][2kcz+1] F(u'_i u'_j)
  double2* uubar;        // [6][n2][kcx+1][2kcz+1] F(u_i u_j), or nullptr
  double2* ubar;         // [3][n2][kcx+1][2kcz+1] F(u_i), or nullptr
  double2* trace;        // trace mode: [n2][kcx+1][2kcz+1] F(u_i u_i) (sum over i)
  const double2* tw;     // f3 plan, float64
  FftPlan plan;
  int n1h, n2, n3, f3;
  int kcx, kcz, K, lstride;
  double scale;          // 1 / (f1 f3)
  int trace_only;        // nonzero: xout holds the trace of the fluctuation squares
};

struct ZinvQArgs {
  const double2* pp;
  FieldsIn u;
  double2* out;          // [n2][9][q3][kcx+1]
  const double2* tw;     // q3 plan
  FftPlan plan;
  int n1h, n2, n3, q3, kcx, kcz, K, lstride;
};

struct XtauArgs {
  const double2* in;     // [n2][9][q3][kcx+1]
  double* tau;           // [6][n2][q3][q1]
  const double2* tw;     // q1 plan
  FftPlan plan;
  int n2, q1, q3, kcx, lstride;
};

// On-the-fly statistics: running sums of |u_i|^2 per mode (mean mode
// excluded) and of the mean profiles
template <typename TP> struct StatsArgs {
  const c2<TP>* u[3];    // u1, u2, u3 spectral [n2][M] (the phase fields)
  double* spec;          // [3][n2][M], += |u_i|^2
  double* mean;          // [2][n2], += U1, U3
  const double* U1;
  const double* U3;
  size_t NP, M;
  int n2;
};
template <typename TP> hipError_t launch_stats(const StatsArgs<TP>& a, hipStream_t st);

template <typename T> hipError_t launch_xfilter(const XfilterArgs<T>& a, size_t lds_bytes, hipStream_t st);
hipError_t launch_zfilter(const ZfilterArgs& a, size_t lds_bytes, hipStream_t st);
hipError_t launch_zinv_q(const ZinvQArgs& a, size_t lds_bytes, hipStream_t st);
hipError_t launch_xtau(const XtauArgs& a, size_t lds_bytes, hipStream_t st);

// ---------------------------------------------------------------- pencils
// Band tables are [n2][7] (row i holds M[i][i-3..i+3]).  LU factors of a
// mode-independent band, for a sweep in either direction: L[i][j] is the
// multiplier of the row at processing distance 3 - j, U[i] = {1/pivot, u1,
// u2, u3}, u_t the entry at distance t on the not-yet-processed side.
struct PencilGeom {
  int n2, n3, n1h, M;         // M = n1h * n3 modes per plane
  double ka, kb;              // 2 pi / lx, 2 pi / lz
  const double *A1, *B1, *A2, *B2;
  const double *L1d, *U1d, *L1u, *U1u, *L2d, *U2d;
  const double *clo, *chi;    // (D1 f)_0 = clo . f, (D1 f)_{n2-1} = chi . f
  const double *quad;         // mass-flux weights
};

// Filtered pressure on the retained modes (Section 3.1): R = (kcx + 1)(2 kcz + 1)
// modes per plane, lane-indexed columns [n2][2R] (two lanes per mode)
struct PressureArgs {
  PencilGeom g;          // compact tables (n2, ka, kb used; M unused)
  const double* uu;      // [6][n2][R] complex F(u_i u_j), pairs 11, 12, 13, 22, 23, 33
  const double* vb;      // [n2][R] complex F(v)
  double* p;             // [n2][R] complex out
  double* T[4];          // lane-indexed scratch [n2][2R]
  double* Q[4];          // mode-indexed scratch [n2][R] (factor rows)
  int R, nz, kcz;
  double nu;
};
hipError_t launch_pressure(const PressureArgs& a, hipStream_t st);

template <typename TP> struct RecoverArgs {
  PencilGeom g;
  const double* v;            // state u2, complex [n2][M]
  const double* om2;          // state omega2
  const double* U1;           // [n2]
  const double* U3;
  TP* out[5];                 // u1, u2, u3, omega1, omega3 (interleaved complex)
  double* S0;                 // lane-indexed scratch, 3 arrays of [n2][2M]
  double* S1;
  double* S2;
  int omega;                  // nonzero: also omega1, omega3 (else out[3], out[4] untouched)
};

template <typename TH, typename TP> struct AdvanceArgs {
  PencilGeom g;
  const TH* H[3];             // H1, H2, H3 (interleaved complex [n2][M])
  TP* ph[5];                  // next sub-step's u1, u2, u3, omega1, omega3 (interleaved complex)
  double* v;                  // state, updated
  double* chi;
  double* om2;
  // histories N_chi, N_omega2 of the previous sub-step, lane-indexed: row i
  // is read at *_rd + i hist_rs and the new one written at *_wr + i hist_ws.
  // hist_rs = 0 where the history has weight zeta = 0 (one finite row is
  // read); hist_ws = 0 where no later sub-step reads it (one junk row).
  const double* nchi_rd;
  const double* nom_rd;
  double* nchi_wr;
  double* nom_wr;
  size_t hist_rs, hist_ws;
  double* S[8];               // scratch, complex [n2][M] (the lane pairs of k_homog: [n2][2 M/2])
  // per-pair [n2][Q] factor tables (k_homog): SU[0..3] the Helmholtz
  // factor rows of this sub-step, SU[4..7] the Poisson ones, each
  // {1/pivot, u1, u2, u3} of the upward / downward factorisation
  const double* SU[8];
  // mean modes
  double* U1;
  double* U3;
  double* nu_old;
  double* nw_old;
  const double* rowsum;       // [2][n2][p3]
  int p3;
  double inv_p1p3;
  double* mean_scr;           // [3][n2][5] solves, then NU, NW, D1 U1, D1 U3 [n2] each
  double* mean_out;           // [0]: mean pressure gradient of the sub-step
  double mass_flux;
  double dt, nu, al, be, ga, ze;
  // per-dt tables of this sub-step (k_homog), one entry per (kx, +-kz) pair
  // q = kx n3/2 + |kz| (Q = M/2 pairs): the SU factor rows are [n2][Q];
  // the homogeneous solution with chi = 1 at wall c is entry c of a (lower,
  // upper) pair
  const double* hc;           // chi_h, [n2][Q][2]
  const double* hm;           // [Q][4]: D1 v_h at (lower, upper) wall for c = 0, then c = 1
  const double* hw;           // [n2][Q][2]: w_c, D1 v_p(wall c) = w_c . r_chi
  // instability guard (common.hpp): every workgroup leaves the state untouched
  // when the fail word is set or the sub-step's CFL (word 0 times dt) is not
  // finite or above cfl_limit; the mean workgroup then records the sub-step
  unsigned* guard;
  double cfl_limit;
  int substep;                // s, for the fail code
};

// Homogeneous solutions of the three sub-steps for a time step dt: the
// Helmholtz step with chi = 1 at one wall and zero forcing, then the Poisson
// step for v, and the wall values of D1 v (influence matrix of Appendix B).
struct HomogArgs {
  PencilGeom g;
  double nu, dt, be[3];
  // tables per (kx, +-kz) pair, Q = M/2 of them (see AdvanceArgs)
  double* hc[3];              // per sub-step, [n2][Q][2]
  double* hw[3];              // per sub-step, [n2][Q][2] (wall-derivative vectors w_c)
  double* hm[3];              // per sub-step [Q][4]
  double* S0;                 // lane-indexed scratch [n2][2M]
  double* S1;
  double* T;                  // lane-indexed scratch [n2][2M] (A2^T E P^-T d_c)
  double* Q[4];               // mode-indexed scratch [n2][M] (factor rows of the transposed solves)
  double* SU[8];              // SU[4..7]: Poisson factor table written here
  double* hu[3][4];           // Helmholtz factor tables of the three sub-steps, written here
};

struct ChiArgs {
  PencilGeom g;
  const double* vin;          // caller's v
  const double* omin;         // caller's omega2
  double* v;                  // state
  double* om2;
  double* chi;
  double* S0;
};

struct InfoArgs {
  PencilGeom g;
  const double* rowcfl;       // [n2][p3]
  int p3;
  const double* U1;
  double dt, nu;
  double* out;                // cfl, mass flux, utau_lo, utau_hi, f (copied), nonfinite flag,
                              // max |divergence| (out[6], as the bits of a non-negative double)
  const double* mean_out;
};

// Divergence of the velocity fields the transforms consume: per mode
// i a u1 + D1 u2 + i b u3 (compact D1 of u2 through the LU of A1); the
// maximum modulus over all modes and nodes is raised into *maxbits (bits of
// a non-negative double, atomicMax).
template <typename TP> struct DivArgs {
  PencilGeom g;
  const TP* u[3];             // u1, u2, u3 interleaved complex [n2][M]
  double* S0;                 // lane-indexed scratch [n2][2M]
  unsigned long long* maxbits;
};
template <typename TP> hipError_t launch_div(const DivArgs<TP>& a, hipStream_t st);

// batched plane phase: descriptors and work lists (context, bx, by, -) in device memory
template <typename T> struct BatchPlan {
  const ZinvArgs<T>* zinv;
  const XpassArgs<T>* xpass;
  const ZfwdArgs<T, T>* zfwd;
  const int4* wz;   // work list of the z passes
  const int4* wx;   // work list of the x pass
  int nz, nx;       // work items
  size_t lds_z, lds_x;
  int mz, mx;       // transform staging (complex values per thread) of the z and x passes
  int rz;           // rows per x-pass workgroup
  int comp;         // nonzero: some channel's plans hold composite radices
};
// Smallest staging size that holds every pass of nlines lines over 256 threads
// (bytes_per_value: 8 for complex float, 16 for complex double); 0 if none.
int staging_for(const FftPlan& pl, int nlines, int bytes_per_value);
template <typename T> hipError_t launch_plane_batch(const BatchPlan<T>& b, hipStream_t st);
template <typename T>
hipError_t launch_advance_batch(const AdvanceArgs<T, T>* d, const int4* w, int nblocks, int n2max, hipStream_t st);

// workgroups of k_advance for M modes per plane (the mean workgroup not counted)
int advance_blocks(int M);
template <typename TP> hipError_t launch_recover(const RecoverArgs<TP>& a, hipStream_t st);
template <typename TH, typename TP> hipError_t launch_advance(const AdvanceArgs<TH, TP>& a, hipStream_t st);
hipError_t launch_homog(const HomogArgs& a, hipStream_t st);
hipError_t launch_chi_from_v(const ChiArgs& a, hipStream_t st);
hipError_t launch_info(const InfoArgs& a, hipStream_t st);
hipError_t launch_convert_d2f(const double* in, float* out, size_t n, hipStream_t st);
hipError_t launch_convert_f2d(const float* in, double* out, size_t n, hipStream_t st);

}  // namespace chn

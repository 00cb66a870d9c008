// Kernel argument blocks shared by the host runtime and the HIP kernels.
// Plain C structs passed by value; pointers are device addresses.
#ifndef SDC_ARGS_H
#define SDC_ARGS_H

typedef long long sdc_i64;
#define SDC_MAXNODE 5

typedef struct {
  double tol;   // Newton stopping tolerance
  double tau;   // pivot threshold of the fixed-order LU
  int maxiter;
  int cap;      // iterations of the fast pass before a zone is deferred (>= maxiter: never)
} NewtonCtl;

// Zones deferred by the fast Newton pass (iteration cap reached, or a pivot
// below tau times its column maximum) and finished by a separate kernel.
typedef struct {
  sdc_i64* z;         // [capacity] zone index
  int* it;            // [capacity] iterations done; -i: the pivot guard stopped iteration i
  double* perr;       // [capacity] size of the last step taken (Newton's stopping test)
  double* x;          // [NX][capacity] current iterate
  double* b;          // [NX][capacity] right-hand side
  double* aux;        // [2 + DIM][capacity] rho, kinetic energy, momenta (transitions)
  unsigned* count;    // entries written
  sdc_i64 capacity;
} DeferQueue;

// Work of one block of the row advection kernel: a run of `slots` (x-row,
// z-chunk) pairs of one periodic grid (the whole domain, or one box).
typedef struct {
  sdc_i64 base;  // zone offset of the grid in the state arrays
  int n0, n1, n2;
  int zc;        // planes per z chunk
  int slot0;     // first slot of the block; slot = y + n1 * chunk
  int nslot;     // slots of the grid: n1 * ceil(n2 / zc)
} RowDesc;

typedef struct {
  const double* U;
  double* A;
  sdc_i64 Z;
  int n[3];
  double idx[3];  // 1 / dx_d
  double gamma;
  double alpha;   // > 0: frozen Rusanov speed
  int slope;      // 0 = central, 1 = MC
  // batched boxes (nbox > 0): zone offsets [nbox+1], extents [nbox][3] and
  // the box holding each 256-zone block's first zone [nblocks]
  int nbox;
  const sdc_i64* box_off;
  const int* box_ext;
  const int* blk_box;
  // row kernel (3D): one descriptor per block
  const RowDesc* rows;
} AdvArgs;

typedef struct {
  sdc_i64 Z;
  double dtm;
  const double* rho;
  const double* b;
  double* x;
  double* R;
  int* iters;
  const void* P;  // NetParams in device memory
  double gm1;
  NewtonCtl ctl;
  unsigned long long* stats;
  DeferQueue q;
} SolveArgs;

typedef struct {
  sdc_i64 Z;
  const double* U;
  double* R;
  const void* P;
  double gm1;
} SourceArgs;

typedef struct {
  sdc_i64 Z;
  int m, M, first;
  double dt, dtm;
  double S[SDC_MAXNODE - 1][SDC_MAXNODE];  // unit-interval integration matrix
  double dtj[SDC_MAXNODE - 1];             // dt_j = (tau_{j+1} - tau_j) dt
  const double* Um;                        // U^{m,(k+1)} (U^n for m = 0)
  const double* Am;                        // A^{m,(k+1)}
  const double* Aold[SDC_MAXNODE];         // A^{j,(k)}     (m = 0, k >= 1)
  const double* Rold[SDC_MAXNODE];         // R^{j,(k)}     (m = 0, k >= 1)
  const double* Cin;                       // C_m           (m >= 1, k >= 1)
  double* Cout[SDC_MAXNODE - 2];           // C_1..C_{M-1}  (m = 0, k >= 1)
  const double* guess;                     // U^{m+1,(k)}, or U^n at k = 0
  double* Uout;
  double* Rout;
  const void* P;
  double gm1;
  NewtonCtl ctl;
  unsigned long long* stats;
  DeferQueue q;
  // split schedule: explicit part and Newton in separate kernels over a zone
  // batch [zbeg, zbeg + zcount); `split` holds [NX + 2][Z]: b, KE, x_e guess
  double* split;
  sdc_i64 zbeg, zcount;
  // fourth-order right-hand-side kernels: the rhs is written to Uout and the
  // Newton guess (reacting vector of U^{m+1,(k)}) to x4 [NX][Z]
  double* x4;
} TransArgs;

// Fourth-order finite volume, zone-per-thread stencil kernels on a periodic
// grid (x fastest).  Face-averaged flux through the face at i+1/2 along `d`
// (flux kernels), its divergence accumulated into A (first: A = -div,
// otherwise A -= div), and the conversions between zone averages and zone
// centres (sign -1: centres from averages, +1: averages from centres) of
// `ncomp` components.
typedef struct {
  const double* U;
  double* F;
  double* A;
  double* Uf;  // face averages along the current direction [NC][Z] (face i+1/2 of every zone)
  sdc_i64 Z;
  int n[3];
  int first;
  double idx;
  double gamma;
} Flux4Args;

typedef struct {
  const double* src;
  double* dst;
  sdc_i64 Z;
  int n[3];
  int ncomp;
  double sign;
} ConvArgs;

// Fourth-order transition pieces around the zone-centre Newton solve.
typedef struct {
  sdc_i64 Z;
  int n[3];
  double dtm;
  double* U;          // [NC][Z] the node's output: the rhs, then U^{m+1} = rhs + dt_m <R>
  double* R;          // [NX][Z] <R>^{m+1}
  double* rho_c;      // [Z] zone-centre density of the rhs
  double* b_c;        // [NX][Z] zone-centre reacting rhs
  const double* R_c;  // [NX][Z] R at the zone-centre root
  const void* P;      // NetParams (source kernel)
  double gm1;
} O4Args;

// Two-level hierarchy (refined patches with subcycling): ghost-zone fills
// of the padded patches from coarse node states, face-flux registers at the
// coarse-fine interfaces, refluxing and average-down.
typedef struct {
  sdc_i64 zf;  // fine zone (index in the concatenated padded patches)
  int pc[3];   // parent coarse zone coordinates
  int sig;     // bit e set: the fine centre is +1/4 coarse zone from the parent's along e, else -1/4
} AmrGhost;

typedef struct {
  double* Uf;                      // fine array [NC][Zf] (state to fill, or A to zero)
  const double* Uc[SDC_MAXNODE];   // coarse node states [NC][Zc]
  double w[SDC_MAXNODE];           // Lagrange weights of the coarse nodes at the fill time
  int nnodes;
  const AmrGhost* list;
  sdc_i64 count;
  sdc_i64 Zc, Zf;
  int nc[3];                       // coarse extents
} AmrFillArgs;

typedef struct {
  sdc_i64 base;  // zone offset of the grid (0: coarse; the box offset for a patch)
  int c[3];      // coordinates of the zone whose i+1/2 face this is
  int n[3];      // grid extents (periodic)
  int d;         // face normal
} AmrFace;

typedef struct {
  const double* U;
  double* reg;   // [NC][count] += coef * F
  const AmrFace* faces;
  sdc_i64 count, Z;
  double coef, gamma, alpha;
  int slope;
} AmrFluxArgs;

typedef struct {
  sdc_i64 zu;     // uncovered coarse zone next to a patch
  sdc_i64 fc;     // its coarse face register
  sdc_i64 ff[4];  // the fine face registers over that face (1, 2 or 4)
  double sign;    // -1: the face is the zone's i+1/2 face, +1: its i-1/2 face
  double h;       // coarse zone width along the face normal
} AmrReflux;

typedef struct {
  sdc_i64 zc;      // covered coarse zone
  sdc_i64 f0;      // its first fine zone
  sdc_i64 sy, sz;  // fine zone strides along y and z
} AmrCover;

typedef struct {
  double* Uc;
  const double* Uf;
  const double* regc;
  const double* regf;
  sdc_i64 Zc, Zf, nregc, nregf;
  const AmrReflux* reflux;
  sdc_i64 nreflux;
  const AmrCover* cover;
  sdc_i64 ncover;
} AmrSyncArgs;

typedef struct {
  double* p;
  sdc_i64 n;
  double v;
} FillArgs;

// Zero several arrays in one launch (the adjoint's accumulators): up to three
// per node (U, A and R adjoints) at the largest node count.
#define SDC_ZERO_MAX (3 * SDC_MAXNODE)
typedef struct {
  double* p[SDC_ZERO_MAX];
  sdc_i64 n[SDC_ZERO_MAX];
  int count;
} ZeroListArgs;

// Adjoint of A (smooth mode: central slopes, frozen Rusanov speed):
// Ubar += (dA/dU)^T Abar, evaluated at U, gather form.
typedef struct {
  const double* U;
  const double* Abar;
  double* Ubar;
  sdc_i64 Z;
  int n[3];
  double idx[3];
  double gamma;
  double alpha;
} AdvVjpArgs;

// Adjoint of one node transition m -> m+1 at iteration k -> k+1, with the
// transposes of its right-hand side assembly fused in.
typedef struct {
  sdc_i64 Z;
  int m, M, first;
  double dt, dtm;
  double S[SDC_MAXNODE - 1][SDC_MAXNODE];
  double dtj[SDC_MAXNODE - 1];
  const double* Uout;      // forward state U^{m+1,(k+1)}
  const double* Uoutbar;   // its adjoint (complete)
  const double* Routbar;   // adjoint of R^{m+1,(k+1)} (complete)
  double* Umbar;           // += rhs bar: adjoint of U^{m,(k+1)} (or of U^n for m = 0)
  double* Ambar;           // += dt_m rhs bar: adjoint of A^{m,(k+1)} (m >= 1)
  double* Aoldbar[SDC_MAXNODE];  // adjoints of A^{j,(k)} (all node 0 when first)
  double* Roldbar[SDC_MAXNODE];  // adjoints of R^{j,(k)}
  const void* P;
  double gm1;
  double tau;
  double* theta_part;      // [nblocks][2 * nreact] partial parameter adjoints
} TransAdjArgs;

// Adjoint of R(U) at U: Ubar += (dR/dU)^T Rbar, parameter partials.
typedef struct {
  sdc_i64 Z;
  const double* U;
  const double* Rbar;
  double* Ubar;
  const void* P;
  double gm1;
  double* theta_part;
} SourceVjpArgs;

// Sum the per-block parameter partials in block order into thetabar (+=).
typedef struct {
  const double* part;
  sdc_i64 nblocks;
  int nparam;
  double* thetabar;
} ThetaReduceArgs;

// y += a * x over n doubles
typedef struct {
  double* y;
  const double* x;
  double a;
  sdc_i64 n;
} AxpyArgs;

#endif

// lks_internal.h -- definitions shared by the kernels and the host layer of
// the MI355X LKS library.  Not part of the public ABI (include/lks.h).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace lks {

// Output tile of the 2D step kernels (threads = TILE_X * TILE_Y); the 3D
// kernels use TILE_X x Tile3<R>::TY.
constexpr int TILE_X = 32;
constexpr int TILE_Y = 8;
constexpr int STEP_THREADS = TILE_X * TILE_Y;
// The 2D adjoint step takes TILE_X x ADJ2D_TY tiles with one thread per node
// of the 2-node halo region (36 x 20 of 768 threads): every load, moment and
// output slot is one thread's.  (The forward keeps 32 x 8 tiles: at 768
// threads per block it holds fewer waves per CU and runs slower.)
constexpr int ADJ2D_TY = 16;
constexpr int ADJ2D_THREADS = 768;
static_assert(ADJ2D_THREADS >= (TILE_X + 4) * (ADJ2D_TY + 4), "one halo-region slot per thread");
// 3D step kernels: one thread per node of the 2-node halo plane.  FP32 takes
// 32 x 16 tiles (36 x 20 halo plane, 768 threads: less halo recomputation);
// FP64 keeps 32 x 8 (36 x 12, 448 threads) so its adjoint, at about 210
// VGPRs, still fits a block on the CU.
template <class R>
struct Tile3 {
  static constexpr int TY = sizeof(R) == 4 ? 16 : 8;
  static constexpr int NT = sizeof(R) == 4 ? 768 : 448;
};
inline int tile3_y(int precision) { return precision == 0 ? 16 : 8; }
// Resident blocks per CU the z-segment lengths of the 3D step kernels are
// chosen for (the grid is about that many times the device's CU count): the
// forward step holds two blocks per CU; the FP32 adjoint (768 threads at up to
// 168 VGPRs) one, the FP64 adjoint two.
constexpr int STEP_RESIDENT_FWD = 2;
inline int step_resident_adj(int precision) { return precision == 0 ? 1 : 2; }
// Compute units and XCDs of the current device (hipDeviceProp_t and
// hipDeviceAttributeNumberOfXccs), read once per plan; MI355X's 256 and 8
// when no device can be queried (plans can be built and validated without
// one).
void device_counts(int* ncu, int* nxcd);
// 3D adjoint step: planes of its LDS ring (4: one barrier per plane; 3: two,
// and less LDS).  FP32 takes 4 (its one block per CU has LDS to spare); FP64
// takes 3 so two blocks fit a CU.
template <class R>
struct AdjRing {
  static constexpr int NR = sizeof(R) == 4 ? 4 : 3;
};
// Threads per block of the map transposes (2D and 3D).
constexpr int MAPADJ_THREADS = 256;
// Objective J2 kernels: one thread per design point (per box node for the seed).
constexpr int J2_THREADS = 256;
// 3D map: most z values per lane the kappa_ref copy is padded for, and the
// value the map uses (one half-wave per analysis column, 32 * MAP_ZPL z
// values per pass).
constexpr int MAP_ZC = 16;
constexpr int MAP_ZPL = 3;
// 3D map: zero padding (design levels) of the z-fastest kappa_ref copy.
constexpr int KZ_PAD = 8;
// 3D forward march with a body slot per step: steps mapped per launch.
constexpr int MAP_BATCH = 8;
// 3D map transpose: design levels per block (short chunks, and long
// ones for FP32 when the design grid has at least 3 x 24 levels).
constexpr int MAPADJ_LCH = 8;
constexpr int MAPADJ_LCH_LONG = 24;
// 2D transfer: a block is a MAP2_TX x MAP2_TY patch of analysis nodes.
constexpr int MAP2_TX = 64, MAP2_TY = 4;

// Device copy of the problem (passed by value to every kernel).
struct Geo {
  int d;
  int n[3];
  int bc[3];
  long long N;
  double A;               // 3/4 - 9 nu / 2
  double uw[3][2][3];
  int D[3];               // design grid incl. margin
  int m[3];
  int margin;
  long long Mtot;
  double xiG[3];          // design centre (geometric centre incl. margin)
  double kmax, q;
  int tlo[3], thi[3];     // target box
  double ndir[3];
  double phi;
  double NTinv;           // 1 / (nt * |T|), 0 for an empty target
  int nt, r_t, r_w;
  double xmin[3], xmax[3], thmin, thmax;
  int org[3];             // tile-grid origin per axis (0 or -1)
  int zseg;               // z planes per block segment (3D adjoint step)
  int zseg_f;             // z planes per block segment (3D forward step)
  int ty3;                // tile height of the step kernels (3D: Tile3<R>::TY; 2D: TILE_Y)
  int prec;               // state precision (0 FP32, 1 FP64)
  int nxcd;               // XCDs of the device (block -> tile order)
  int rot;                // 0: one angle about z; 1: three angles (3D)
  int mw;                 // motion row width: 8, or 12 with three angles
  int nmc;                // motion components: x, y, z and the angles (4 or 6)
  double tmin[2], tmax[2]; // rot = 1: ranges of the angles about x and y
  int obj;                // objective: 0 J1, 1 J2
  double j2s[3];          // J2 normalisations 1/(nt M), 1/((x2max - x2min) M),
                          // 1/(2 pi l_m M), M = inner design points
  double j2w[2];          // J2 weights w_d, w_t
};

// Inner design points (no margin): the size of gamma.
__host__ __device__ inline long long inner_points(const Geo& g) {
  long long M = 1;
  for (int a = 0; a < g.d; ++a) M *= g.m[a];
  return M;
}

// Blocks of the 2D map transpose (a 16 x 16 patch of design points each).
__host__ __device__ inline int mapadj_blocks_2d(const Geo& g) {
  return ((g.D[0] + 15) / 16) * ((g.D[1] + 15) / 16);
}

// Support box of the body at one step, in unwrapped analysis coordinates;
// the body buffers are laid out with fixed strides sx, sy (max extents).
struct Box {
  int lo[3];
  int ext[3];
  int sx, sy;
  long long vol;  // size of one plane of the body buffers (sx * sy * max ext z)
};

// Per-step body data computed on the device by the prelude: rigid motion
// (centre, velocity, cos/sin of the angle, angular velocity) and the support
// box.  Step kernels read it, so their launch arguments do not change from
// call to call (the time loops can be captured once and replayed).
struct StepInfo {
  double xg[3], ug[3], c, s, om;
  int lo[3], ext[3], flag, pad;
  // rotation matrix and its time derivative (row major): with three angles
  // R = Rz(th3) Ry(th2) Rx(th1) and Rd = sum_k om_k dR/dth_k; about z alone
  // the same for R(theta)
  double R[9], Rd[9];
  double th[3], om3[3];  // the angles and their rates (about z alone: th[2], om3[2])
};

// Rotation about coordinate axis ax by angle a, differentiated `order` times
// in a (0, 1 or 2), row major.
__host__ __device__ inline void axis_rot(int ax, double a, int order, double* M) {
  for (int k = 0; k < 9; ++k) M[k] = 0.0;
  const double c = cos(a), s = sin(a);
  double cn = c, sn = s;
  if (order == 1) {
    cn = -s;
    sn = c;
  } else if (order == 2) {
    cn = -c;
    sn = -s;
  }
  const int i = (ax + 1) % 3, j = (ax + 2) % 3;
  M[ax * 3 + ax] = order == 0 ? 1.0 : 0.0;
  M[i * 3 + i] = cn;
  M[i * 3 + j] = -sn;
  M[j * 3 + i] = sn;
  M[j * 3 + j] = cn;
}
// Rz(th[2]) Ry(th[1]) Rx(th[0]), each factor differentiated o[k] times.
__host__ __device__ inline void euler_mat(const double* th, const int* o, double* M) {
  double X[9], Y[9], Z[9], ZY[9];
  axis_rot(0, th[0], o[0], X);
  axis_rot(1, th[1], o[1], Y);
  axis_rot(2, th[2], o[2], Z);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = 0.0;
      for (int k = 0; k < 3; ++k) v += Z[i * 3 + k] * Y[k * 3 + j];
      ZY[i * 3 + j] = v;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = 0.0;
      for (int k = 0; k < 3; ++k) v += ZY[i * 3 + k] * X[k * 3 + j];
      M[i * 3 + j] = v;
    }
}
// Angles and rates of a motion row (8 or 12 values): about z alone the
// angle and rate sit in th[2], om[2].
__host__ __device__ inline void row_angles(int mw, const double* m, double th[3], double om[3]) {
  if (mw == 12) {
    for (int k = 0; k < 3; ++k) {
      th[k] = m[6 + k];
      om[k] = m[9 + k];
    }
  } else {
    th[0] = th[1] = om[0] = om[1] = 0.0;
    th[2] = m[6];
    om[2] = m[7];
  }
}
// Rotation and rate matrices of a motion row.
__host__ __device__ inline void row_rotation(int mw, const double* m, double* R, double* Rd) {
  double th[3], om[3];
  row_angles(mw, m, th, om);
  const int o0[3] = {0, 0, 0};
  euler_mat(th, o0, R);
  for (int k = 0; k < 9; ++k) Rd[k] = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (om[a] == 0.0) continue;
    int o[3] = {0, 0, 0};
    o[a] = 1;
    double D[9];
    euler_mat(th, o, D);
    for (int k = 0; k < 9; ++k) Rd[k] += om[a] * D[k];
  }
}

// Standard velocity sets with opposite directions in consecutive pairs
// (rest direction first).
template <int Q>
struct Lat;
template <>
struct Lat<9> {
  static constexpr int d = 2;
  static constexpr int c[9][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                  {1, 1, 0},  {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}};
  static constexpr double w[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};
template <>
struct Lat<15> {
  static constexpr int d = 3;
  static constexpr int c[15][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                                   {0, 0, 1},   {0, 0, -1},  {1, 1, 1},   {-1, -1, -1},
                                   {-1, 1, 1},  {1, -1, -1}, {1, -1, 1},  {-1, 1, -1},
                                   {1, 1, -1},  {-1, -1, 1}};
  static constexpr double w[15] = {2.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,
                                   1.0 / 9,  1.0 / 9,  1.0 / 72, 1.0 / 72, 1.0 / 72,
                                   1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72};
};

// Profiling: when `start` is set, the next step or map launch carries this
// event pair in its dispatch (hipExtLaunchKernelGGL), so the pair times the
// kernel itself; the launch clears it.  Thread-local, host side only.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents& launch_events();

// ---- launch wrappers (lks_kernels.hip) ----
struct FwdArgs {
  const void* in;
  void* out;
  const void* bk;    // kappa on the body box (nullable: no body)
  const void* bu;    // body velocity planes [d][box.vol]
  Box box;
  double* opart;     // [blocks][2] objective partials (nullable)
  int* flags;        // [0]: instability flag
  int lazy_wall;     // 1: wall-node pressures of `in` follow the wall rule
  const StepInfo* si; // nullable: step box taken from the device table
};
struct AdjArgs {
  const void* lam;      // dJ/d state(n)
  void* lam_prev;       // dJ/d state(n-1)
  const void* u_prev;   // state(n-1)  (velocity planes read)
  const void* u_cur;    // state(n)    (velocity planes read; seed and kappa bar)
  const void* bk;       // body fields on the box (nullable)
  const void* bu;
  void* bkbar;          // dJ/dkappa on the box
  void* bubar;          // dJ/du_s on the box [d][box.vol]
  Box box;
  const double* seed;   // dJ (device, nullable -> no objective seed)
  const double* E;      // mean of n.u from the forward (device)
  const StepInfo* si;   // nullable: step box taken from the device table
  // Paper-literal ALKS instead of the exact transpose (both null: exact).
  // The adjoint velocity state then has two parts: lam holds the whole
  // vector of the adjoint equilibrium, xin its raw first-moment part
  // 3 u~ ([d][N], read on body-box nodes only), on which alone the
  // Brinkman source acts; xout receives the raw part of step n - 1 on the
  // body box of step n - 1 (si_next; nullable: nowhere, no step reads it).
  const void* xin;
  void* xout;
  const StepInfo* si_next;
  int xall;  // ALKS: store the raw part at every node (the sweep's last step)
  // Objective J2: seed on the fluid velocity on the body box ([2][box.vol],
  // box-indexed like bk; nullable), applied where the J1 seed would be.
  const void* j2s;
  // ALKS (nullable): the state of level n - 1 in the paper's variables,
  // p~ [N], u~ [d][N] and the symmetric s~ [d(d+1)/2][N] ((xx, yy, xy) in
  // 2D, (xx, yy, zz, xy, xz, yz) in 3D), written at every node; the sweep's
  // last step sets it for the periodic approximation's carry.
  void* mout;
};

int step_blocks(const Geo& g);
// Planes of the ALKS state (p~, u~, symmetric s~).
inline int alks_carry_planes(int d) { return 1 + d + d * (d + 1) / 2; }
// ALKS carried state (p~, u~, s~ at the last level, layout as AdjArgs::mout)
// and that level's flow state st -> the adjoint state the reverse sweep
// starts from: lam = (-3 p~, -V) and the raw first-moment part X = -3 u~.
hipError_t launch_alks_carry_in(const Geo& g, int precision, const void* carry, const void* st,
                                void* lam, void* X, hipStream_t s);
hipError_t launch_forward_step(const Geo& g, int precision, const FwdArgs& a, hipStream_t s);
hipError_t launch_adjoint_step(const Geo& g, int precision, const AdjArgs& a, hipStream_t s);
size_t kz_bytes(const Geo& g, int ext2max, int precision);
hipError_t launch_kref_t(const Geo& g, int precision, const void* kref, void* kt, hipStream_t s);
// nsteps > 1 (3D, rotation about z, per-step table): consecutive steps from
// si, body slots bstride values apart.
hipError_t launch_map(const Geo& g, int precision, const void* kref, void* kzbuf, int ext2max,
                      const double* mot8_host, const StepInfo* si, const Box& box, void* bk,
                      void* bu, int full_grid, hipStream_t s, int nsteps = 1,
                      long long bstride = 0);
int mapadj_blocks(const Geo& g);
// Map transposes of consecutive steps in one launch (blockIdx.y = step
// within the batch): step k reads si[k] and its body adjoint advanced by
// k * body values, and writes its kappa_ref partials and motion partials
// advanced by k * kref and k * mpart values.
struct StepBatch {
  long long body, kref, mpart;
};
hipError_t launch_map_adjoint(const Geo& g, int precision, const void* kref,
                              const double* mot8_host, const StepInfo* si, const Box& box,
                              const void* bkbar, const void* bubar, double* kref_bar, int overwrite,
                              double* mpart, hipStream_t s, int nsteps = 1,
                              StepBatch sb = StepBatch{0, 0, 0});
// kref_bar[k] += part[j * M + k] for j = n - 1 down to 0, one at a time.
// Objective J2 (2D): blocks of the per-design-point kernels; the step sums
// of state st after step si added into jacc [j2_blocks][3]; (J2, F_L, F_D)
// from them; the reverse-step seeds on the body box and the direct terms of
// nsteps consecutive steps (see the kernels).
int j2_blocks(const Geo& g);
hipError_t launch_j2_forward(const Geo& g, int precision, const void* kref, const StepInfo* si,
                             const void* st, double* jacc, hipStream_t s);
// 2D: the LKS step of `a`, the transfer of step msi into the body fields
// (bk, bu on the box; not the step's own; msi null: none) and, when jst is
// non-null, the J2 step sums of state jst after step jsi, in one launch.
hipError_t launch_forward_step_map(const Geo& g, int precision, const FwdArgs& a,
                                  const void* kref, const StepInfo* msi, const Box& box, void* bk,
                                  void* bu, const StepInfo* jsi, const void* jst, double* jacc,
                                  hipStream_t s);
// 2D: the transfer of step si into the body fields (bk, bu on the box) and
// the J2 step sums of state jst after step jsi, in one launch.
hipError_t launch_map_j2(const Geo& g, int precision, const void* kref, const StepInfo* si,
                         const Box& box, void* bk, void* bu, const StepInfo* jsi, const void* jst,
                         double* jacc, hipStream_t s);
hipError_t launch_j2_final(const Geo& g, const double* jacc, double* J3, hipStream_t s);
hipError_t launch_j2_seed(const Geo& g, int precision, const void* kref, const StepInfo* si,
                          const Box& box, const double* dJ, void* js, int nsteps, hipStream_t s);
hipError_t launch_j2_adjoint(const Geo& g, int precision, const void* kref, const StepInfo* si,
                             const void* st0, long long sstride, const double* dJ, double* kpart,
                             long long kstride, double* mpart, long long mstride, int slot0,
                             int nsteps, hipStream_t s);
hipError_t launch_kref_accum(long long M, int n, const double* part, double* kref_bar,
                             hipStream_t s);
hipError_t launch_steps(const Geo& g, const double* mot, StepInfo* tab, int* info, hipStream_t s);
hipError_t launch_kappa_ref(const Geo& g, int precision, const double* gamma, void* kref,
                            hipStream_t s);
hipError_t launch_design_filter(const Geo& g, const double* gamma, double radius, double beta,
                                double eta, double* phys, hipStream_t s);
hipError_t launch_design_filter_adjoint(const Geo& g, const double* gamma, double radius,
                                        double beta, double eta, const double* gbar, double* work,
                                        double* out, hipStream_t s);
// Most inner design points the allocation-free chain rule takes (its
// scratch is a fixed device array of this many doubles: 16 MiB).
constexpr long long NOALLOC_MAX_POINTS = 1LL << 21;
// Device address of that array on the current device (looked up once per device).
hipError_t noalloc_scratch(double** out);
hipError_t launch_constraints(const Geo& g, const double* phys, const double* chi,
                              const double* psi, double vmax, double omax, double pw,
                              double* Gout, double* dG1, double* dG2, double* dG3_dpsi, double* mot,
                              double* mbar, double* den, double* dchi_scratch, hipStream_t s);
hipError_t launch_motion(const Geo& g, const double* chi, const double* psi, double* mot,
                         hipStream_t s);
hipError_t launch_boxes(const Geo& g, const double* mot, int* boxes, int* info, hipStream_t s);
hipError_t launch_objective_final(const Geo& g, const double* opart, int nblk, double* J3,
                                  hipStream_t s);
hipError_t launch_sens(const Geo& g, int precision, const double* gamma, const double* kref_bar,
                       const double* mpart, int nblk, double* mbar, double* den_t, double* den_w,
                       double* dgamma, double* dchi, double* dpsi, hipStream_t s);
hipError_t launch_state_init(const Geo& g, int precision, void* st, hipStream_t s);
hipError_t launch_reduce_parts(const Geo& g, const double* part, int nblk, double* out8,
                              hipStream_t s);
hipError_t launch_wall_fixup(const Geo& g, int precision, void* st, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// flag[0] = 1 where the n doubles of a and b differ bitwise (flag untouched otherwise).
hipError_t launch_differ(const double* a, const double* b, long long n, int* flag, hipStream_t s);

// ---- batched 2D launches: one launch covers the same step of up to
// BATCH_MAX independent instances; instance k owns blocks
// [start[k], start[k+1]) (starts are multiples of 8, the extra blocks of an
// instance exit at once).  Geo lives in each instance's workspace.
constexpr int BATCH_MAX = 16;
struct MapArgs {
  const void* kref;
  const StepInfo* si;
  Box box;
  void* bk;
  void* bu;
  int bxn;  // blocks along x of one box row
};
struct MapAdjArgs {
  const void* kref;
  const StepInfo* si;
  Box box;
  const void* bkbar;
  const void* bubar;
  double* kref_bar;
  double* mpart;
  int overwrite;
  StepBatch sb;  // strides between the steps of a launch over several steps
};
template <class A>
struct Batch {
  const Geo* geo[BATCH_MAX];
  A a[BATCH_MAX];
  int start[BATCH_MAX + 1];
  int count;
};
static_assert(sizeof(Batch<AdjArgs>) < 4000 && sizeof(Batch<FwdArgs>) < 4000 &&
                  sizeof(Batch<MapArgs>) < 4000 && sizeof(Batch<MapAdjArgs>) < 4000 &&
                  sizeof(Batch<FwdArgs>) + sizeof(Batch<MapArgs>) < 4000,
              "batched launch arguments must fit the kernel argument buffer");
int step_blocks_2d(const Geo& g);
int adj2d_blocks(const Geo& g);  // tiles of the 2D adjoint step  // tiles of the 2D step kernels
int map_blocks_2d(const Box& bmax, int* bxn);
hipError_t launch_forward_step_batch(int precision, const Batch<FwdArgs>& b, hipStream_t s);
// Step n of every instance and the transfer of step n + 1 (mb) in one launch.
hipError_t launch_forward_step_map_batch(int precision, const Batch<FwdArgs>& fb,
                                        const Batch<MapArgs>& mb, hipStream_t s);
hipError_t launch_adjoint_step_batch(int precision, const Batch<AdjArgs>& b, hipStream_t s);
hipError_t launch_map_batch(int precision, const Batch<MapArgs>& b, hipStream_t s);
hipError_t launch_map_adjoint_batch(int precision, const Batch<MapAdjArgs>& b, hipStream_t s,
                                    int nsteps = 1);
__host__ __device__ void body_box(const Geo& g, const double* m8, int* out);
// StepInfo of one motion row (box included).
__host__ __device__ void step_info(const Geo& g, const double* mrow, StepInfo& si);

}  // namespace lks

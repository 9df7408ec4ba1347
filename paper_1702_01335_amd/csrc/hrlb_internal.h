// Internal declarations shared by the host C ABI (capi.cpp), the host quadrature
// (quadrature.cpp) and the device kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace hrlb {

constexpr int NX_MAX = 8;    // largest half-range expansion order on x
constexpr int NYZ_MAX = 15;  // largest full-range expansion order on y, z (Q <= 16)
constexpr int QYZ_MAX = 16;
constexpr int QX_MAX = 128;
constexpr int REC_HEAD = 16;  // scalars at the head of a per-node closure record
constexpr int NMOM = 13;         // moment sums per node (n, n u, the second moments, the energy fluxes)
constexpr int PART_STRIDE = 16;  // doubles per node row of the closure's summed moments (13 + n, u_x, T)
// Moment partials in HBM: per instance, 16-node group and 64-velocity block, NMOM lines
// of the group's 16 nodes (moment-major, so a moment of a whole group is one 128-byte line)
constexpr int PART_GROUP = NMOM * 16;
constexpr int part_groups(int S) { return (S + 15) >> 4; }
constexpr int MAX_WAVES = 4;   // waves per stage-kernel workgroup (LDS: 8.3 KB per wave, 12.4 KB with several)
// 64-velocity blocks of the moment-multiplier table: those of V, plus the whole idle waves
// a workgroup of up to MAX_WAVES waves can hold past V
constexpr int ptab_blocks(int V) { return (V + 63) / 64 + MAX_WAVES - 1; }

// Host quadrature tables (double, rounded from long double).  In the reduced (phi, chi)
// model the z axis is replaced by the two reduced distributions: Qz = 2 "components"
// (0: phi, 1: chi), pz = {0, 0}, and the z factor of the equilibrium is {1, T}.
struct QuadTables {
  int Qx, Nx, Qy, Ny, Qz, Nz;
  int reduced;
  std::vector<double> px, wx;    // 2 Qx, ascending
  std::vector<double> py, wy;    // Qy
  std::vector<double> pz, wz;    // Qz
  std::vector<double> phix;      // [Qx][Nx+1]: w_m h_l(p_m) / gamma_l, positive nodes m
  std::vector<double> cx;        // [Nx+1][Nx+1]: monomial coefficients of monic h_l
  std::vector<double> phiy;      // [Qy][Ny+1]: w_j He_l(p_j) / l!
  std::vector<double> phiz;      // [Qz][Nz+1]
};

int build_quadrature(int Qx, int Nx, int Qy, int Ny, int Qz, int Nz, QuadTables& qt);

// Per-instance constants on the device (doubles, fixed layout).
struct InstDev {
  double dt, kn, omega, suth, pr, n0, T_w, u_w;
  double wall_den;   // sum_{p_x<0} p_x F^eq_w / n_w   (filled on the device)
  double ex[6];      // Lagrange weights: ghost S from S-1,S-2,S-3 and ghost S+1 from S,S-1,S-2 (0-based)
  double law;        // 0 power, 1 Sutherland, 2 low Mach
  double collisionless;
  double pad;
};
static_assert(sizeof(InstDev) == 18 * 8, "InstDev layout");

// Device pointers of a sim (all carved out of the caller's work and state buffers).
struct DevPtrs {
  // velocity set tables
  const double* px;   // [2Qx]
  const double* py;   // [Qy]
  const double* pz;   // [Qz]
  const double* phix; // [Qx][Nx+1]
  const double* cx;   // [Nx+1][Nx+1]
  const double* phiy; // [Qy][Ny+1]
  const double* phiz; // [Qz][Nz+1]
  double* ptab;       // moment multipliers in MFMA operand order, [ptab_blocks(V)][8][64][2] (filled on the device)
  // per instance
  InstDev* inst;      // [B]
  double* inv_dx;     // [B][S]
  double* g_rest;     // [B][V]  discrete equilibrium at rest per unit density
  double* g_wall;     // [B][V]  wall Maxwellian per unit density
  // per step / stage
  double* partials;   // [B][part_groups(S)][nvb][NMOM][16] (16-node groups, moment lines)
  double* rec;        // [B][S][rec_len]
  double* nw;         // [B]
  double* resid_part; // [B][nres][2]
  double* resid;      // [B]
  int* flags;         // [B]
  double* junk;       // [256]: store target of stage-kernel lanes beyond V (never read)
  // populations
  double* F[3];       // three [B][S][V] arrays
};

struct Shape {
  int Qx, Nx, Qy, Ny, Qz, Nz;
  int V, QyQz, S, B;
  int scheme;
  int rec_len;        // REC_HEAD + 2 Qx + Qy Qz, rounded up to a multiple of 16 (whole lines)
  int reduced;        // 1: the paper's reduced (phi, chi) model, Qz = 2 components
  int pad;
};

// One uniform group (one sim) inside a batch, as the batched kernels see it.
struct GroupDesc {
  Shape sh;
  DevPtrs d;
  int nvb, nch, cs;        // stage-kernel tiling (waves per block is the batch's)
  int node_blocks, nb;     // closure work split: node blocks of nb nodes, then B wall items
  int pad[3];
};

// Work-buffer carve-up; returns the total bytes and fills offsets.
struct WorkLayout {
  size_t px, py, pz, phix, cx, phiy, phiz, ptab, inst, inv_dx, g_rest, g_wall, partials, rec, nw, resid_part,
      resid, flags, junk, total;
  int nvb_max, nres_max;
};
WorkLayout work_layout(const Shape& sh);

// Kernel launchers (kernels.hip).  Every launcher returns a hipError_t cast to int.
// record the message returned by hrlb_last_error() for this thread; returns code
int set_error(int code, const char* msg);

int launch_setup_tables(const Shape& sh, const DevPtrs& d, void* stream);
int launch_init_state(const Shape& sh, const DevPtrs& d, const double* perturb, double eps, void* stream);
int launch_fm_state(const Shape& sh, const DevPtrs& d, void* stream);
int launch_seed(const Shape& sh, const DevPtrs& d, const double* tab, int preserve_mass, void* stream);
int launch_clear_flags(const Shape& sh, const DevPtrs& d, void* stream);
int launch_partials(const Shape& sh, const DevPtrs& d, const double* F, int cells, int waves, void* stream);
int launch_closure(const Shape& sh, const DevPtrs& d, const double* Fin, int nvb, double* mom_out, void* stream);
int launch_stage(const Shape& sh, const DevPtrs& d, int stage, const double* Fin, const double* Fl, double* Fout,
                 int cells, int waves, void* stream);
int launch_residual(const Shape& sh, const DevPtrs& d, int nres, void* stream);

// batched launches over several groups: tiles are int4 (group, instance, vblock, chunk),
// closure items int2 (group, block); counts live in device memory so a captured graph
// keeps working when the tables are rewritten
int launch_batch_stage(int stage, const GroupDesc* groups, const void* tiles, const int* ntiles, int grid, int waves,
                       size_t lds_bytes, void* stream);
int launch_batch_closure(int stage, const GroupDesc* groups, const void* items, const int* nitems, int grid,
                         size_t lds_bytes, void* stream);
size_t stage_lds_bytes_for(int waves);
size_t closure_lds_bytes_for(const Shape& sh, int nb);
constexpr int CL_NODES = 16;  // most nodes per closure block
int closure_nodes_for(int total_nodes);
int batch_closure_blocks_per_cu(size_t lds_bytes);  // resident batch-closure blocks per CU

// bytes of the fixed per-GPU work array of hrlb_step_noalloc (HRLB_SCRATCH_BYTES in hrlb.h)
constexpr size_t SCRATCH_BYTES = (size_t)32 << 20;
// device address of that array on the current device (looked up once per device); returns
// a hipError_t cast to int
int scratch_pointer(void** out);

}  // namespace hrlb

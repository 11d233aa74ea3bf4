// Internal declarations shared by the host side of the C ABI and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtmm.h"

// Threads per workgroup of every cell-parallel kernel (four 64-wide waves).
#define RT_BLOCK 256

struct rt_mesh {
  int device;
  int64_t N, F, H;  // cells, faces, half-faces (= 2F)
  int32_t k_max, flags;
  double box;
  // geometry resident on the device
  double *vol0;       // [N] geometric volumes (gradient estimator)
  double *D;          // [N] volume rate sum_faces A (w~.n), outward positive
  double *wn;         // [F] face normal speed w~.n
  int32_t *row_ptr;   // [N+1] half-faces of cell i are [row_ptr[i], row_ptr[i+1])
  int32_t *hf_nbr;    // [H] the other cell of each half-face
  int32_t *hf_face;   // [H] face id f for the face's first cell, -(f+1) for its second
  double4 *hf_an64;   // [H] (A n_out, A (w~.n)_out), FP64
  float4 *hf_an32;    // [H] same, FP32
  // reconstruction geometry (RT_MESH_PLM): per half-face, from the owning cell's side
  double4 *hf_gp64;   // [H]: (A c/d + A/2 n_g, 0), the neighbour's weight in the gradient
  double4 *hf_rel64;  // [H][2]: (r~ - s_self, r~ - s_nbr.x), (r~ - s_nbr.y, .z, -, -)
  float4 *hf_gp32;
  float4 *hf_rel32;
  double4 *gb64;      // [N]: (sum over the cell's faces of A/2 n_g - A c/d, 0), its own weight
  float4 *gb32;
  // scratch
  void *I_half;       // [N][k_max] doubles (RT_MESH_PLM), used in either precision
  void *grad;         // RT_MESH_PLM, 4 N k_max doubles: FP32 (I_half, limited gradient) per cell
                     // and angle [N][K][4]; FP64 the limited gradient [N][3][K]
  void *lam_star;     // [N][k_max] doubles (RT_MESH_ADJOINT)
  double *red;        // reduction partials, RT_NDIAG * n_red_blocks doubles
  double *red_mid;    // first fold of the partials, RT_NDIAG * RT_BLOCK doubles
  int64_t n_red_blocks;
  int32_t lds_max;    // LDS bytes a workgroup may use on the upload's device
  int32_t hf_cap16;   // most half-faces of any 16 consecutive cells (workgroups of 16 cells)
  int32_t hf_cap32;   // same for 32 consecutive cells
  int32_t hf_cap64;   // same for 64 consecutive cells
  // per workgroup of 16 / 32 / 64 consecutive cells, the cells ordered by face count:
  // lane group g of the workgroup starting at cell c0 takes cell c0 + wg_order*[c0 + g], so
  // each wave holds cells of similar face counts and its face loop pads less
  uint8_t *wg_order16, *wg_order32, *wg_order64;
};

// ------------------------------------------------------------------------------------------
// launch helpers implemented in the kernel files; all return hipError_t of the launch
// ------------------------------------------------------------------------------------------

struct rt_step_args {
  int64_t N;
  int K;
  const int32_t *row_ptr;
  const int32_t *hf_nbr;
  const void *hf_an;   // double4* or float4*
  const void *hf_rel;  // PLM only
  const double *D;
  const double *dirs;
  const double *W;
  const void *I_in;    // intensities read by transport (start-of-step charges)
  const void *I_half;  // PLM stage 2: half-step intensities (face states)
  const void *grad;    // PLM stage 2: FP32 (I_half, limited gradient) [N][K][4]; FP64 gradient [N][3][K]
  void *I_out;
  void *I_star_out;    // upwind with source: when set, the transported intensities (the
                       // source's input) are stored here as well
  const double *vol_in;
  double *vol_out;
  const double *rho;
  double *mom;
  double *etot;
  const double *kP;
  const double *kJ;
  const double *ks;
  double *T_out;
  double *src_tape_out;  // taped upwind step: per-cell source values for the reverse
                         // ([N][RT_SRC_TAPE]), written when set
  // modes 4 and 5 (reverse of the source of step n)
  const void *I_next;       // the output intensities of step n
  const double *src_tape;   // its source tape
  double *lamE, *lamM;      // dL/d(E_g, m)^{n+1} in, dL/d(E_g, m)^n out
  double *dkP, *dkJ;        // incremented when set (may be one array)
  double c_red, c_light, a_rad, cv, dt;
  double inv_c;       // 1 / c
  double e_gain;      // 4 pi c / cbar: gas energy per unit of sum W (I - I')
  double m_gain;      // 4 pi / cbar: gas momentum per unit of sum W n (I - I')
  double a_4pi;       // a / 4 pi
  int paired;        // rt_pair_kind of the angle layout
  int hf_cap;        // LDS staging slots of the launched kernel (set at dispatch)
  int lds_max;       // LDS bytes a workgroup may use
  int hf_cap16, hf_cap32, hf_cap64;  // half-faces of the largest range of 16 / 32 / 64 cells
  const uint8_t *wg_order16, *wg_order32, *wg_order64;  // cell order within workgroups
  const uint8_t *wg_order;                              // the one of the launched kernel
  int do_transport;  // 0: source only (in place), 1: upwind, 2: reconstructed (PLM stage 2),
                     // 3: transpose of upwind transport (adjoint), 4: transpose of step n + 1
                     // then the source reverse of step n, 5: source reverse of step n only
  int do_source;
  int write_gas;
};

// Per-cell values the taped forward step stores for the reverse ([N][RT_SRC_TAPE] doubles):
// the source solve's 1 / sum W Gamma^-2, S1, SG, SI, 1 / D and T^{n+1}, then the
// start-of-step volume and gas momentum (3).
enum { RT_TAPE_IQ = 0, RT_TAPE_S1, RT_TAPE_SG, RT_TAPE_SI, RT_TAPE_ID, RT_TAPE_T, RT_TAPE_V, RT_TAPE_M };
static_assert(RT_TAPE_M + 3 == RT_SRC_TAPE, "tape layout");

hipError_t rt_launch_face_speed(const double *gen, const double *mesh_vel, const int32_t *face_cells,
                                const int8_t *face_shift, const double *face_normal, const double *face_centroid,
                                double box, int64_t F, double *wn, hipStream_t s);
hipError_t rt_launch_half_faces(rt_mesh *m, const int32_t *face_cells, const double *face_area,
                                const double *face_normal, const double *face_centroid, const double *gen,
                                const double *com, const int8_t *face_shift, hipStream_t s);
hipError_t rt_launch_gradient_base(rt_mesh *m, const int32_t *face_cells, const double *face_area,
                                   const double *face_centroid, const double *gen, const int8_t *face_shift,
                                   hipStream_t s);
hipError_t rt_launch_volume_rate(rt_mesh *m, hipStream_t s);

// Lane layout of the step kernel for K angles: (lanes per cell << 8) | angles per lane.
// Antipodal sets (either order) with K/2 a multiple of 8 (K/8 in 2..12) or of 4 (K/4 in
// {2, 6, 10}) use the paired kernel; everything else 16 lanes (K a multiple of 16 or above
// 64) or 8.
// The paired layout for K, or 0 when the paired kernel has none (the general kernel
// then serves the set even if it is antipodal).
static inline int rt_paired_lanes(int K) {
  if (K % 2 == 0) {
    const int half = K / 2;
    if (half % 8 == 0 && K / 8 >= 2 && K / 8 <= 12) return (8 << 8) | (K / 8);
    if (half % 4 == 0 && (K / 4 == 2 || K / 4 == 6 || K / 4 == 10)) return (4 << 8) | (K / 4);
  }
  return 0;
}
// The paired lane layout of the kernels for an angle layout: 1 (antipode at k + K/2),
// 2 (antipode at k + 1, pairs adjacent), 0 (none).
static inline int rt_pair_kind(int layout) {
  return layout == RT_ANGLES_ANTIPODAL ? 1 : layout == RT_ANGLES_ANTIPODAL_ADJACENT ? 2 : 0;
}
static inline int rt_step_lanes(int K, int paired) {
  if (paired && rt_paired_lanes(K)) return rt_paired_lanes(K);
  if (K % 16 == 0 || K > 64) return (16 << 8) | ((K + 15) / 16);
  return (8 << 8) | ((K + 7) / 8);
}

hipError_t rt_launch_step(const rt_step_args &a, int dtype, hipStream_t s);
hipError_t rt_launch_gradient(const rt_mesh *m, int K, const void *I, void *grad, int dtype, bool packed,
                              hipStream_t s);

struct rt_adj_args {
  int64_t N;
  int K;
  const int32_t *row_ptr;
  const int32_t *hf_nbr;
  const void *hf_an;
  const double *D;
  const double *dirs;
  const double *W;
  const void *I_star;
  const double *vol_n;
  const double *rho;
  const double *mom;
  const double *etot;
  const double *kP;
  const double *kJ;
  const double *ks;
  void *lamI;       // in: dL/dI^{n+1}; out: dL/dI^n
  void *lam_star;   // scratch: dL/dI*
  double *lamE;
  double *lamM;
  double *dkP;
  double *dkJ;
  double c_red, c_light, a_rad, cv, dt;
};
hipError_t rt_launch_adjoint(const rt_adj_args &a, int dtype, hipStream_t s);

// Multigroup source (group-major intensities [G][N][K], opacities [G][N]).
#define RT_G_MAX 16
struct rt_mg_args {
  int64_t N;
  int K, G;
  int paired;
  const double *dirs;
  const double *W;
  const double *Wg;  // [G] group weights
  void *I;
  const double *rho;
  double *mom;
  double *etot;
  const double *kP, *kJ, *ks;
  double *T_out;
  double c_red, c_light, a_rad, cv, dt;
  double inv_c, e_gain, m_gain, a_4pi;
};
hipError_t rt_launch_source_mg(const rt_mg_args &a, int dtype, hipStream_t s);

// Source with power-law temperature-dependent opacities.
struct rt_kT_args {
  int64_t N;
  int K;
  const double *dirs;
  const double *W;
  void *I;
  const double *rho;
  double *mom;
  double *etot;
  const double *kP0, *kJ0, *ks;
  double *T_out;
  double T_ref, bP, bJ;
  double c_red, c_light, a_rad, cv, dt;
  double e_gain, m_gain;
  int paired;  // rt_pair_kind of the angle layout
};
hipError_t rt_launch_source_kT(const rt_kT_args &a, int dtype, hipStream_t s);

// Marked cells (boundary / emitter) resident on the device.
struct rt_marked {
  int64_t n_cells;  // cell count of the mesh the set was made for
  int64_t n;        // marked cells
  int32_t *cell, *kind;
  double *T_eff, *dir, *cos_open;
  double tau;
};

struct rt_marked_args {
  int64_t n;
  int K;
  const int32_t *cell;
  const int32_t *kind;
  const double *T_eff;
  const double *dir;
  const double *cos_open;
  const double *dirs;
  const double *W;
  void *I;
  const double *rho;
  double *mom;
  double *etot;
  const double *kP;
  double f;  // min(dt / tau, 1)
  double dt, a_rad, c_red, c_light;
};
hipError_t rt_launch_marked(const rt_marked_args &a, int dtype, hipStream_t s);

hipError_t rt_launch_flux_loss(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light,
                               const void *I, const double *face_weight, double *loss, void *seed, int dtype,
                               hipStream_t s);
// The loss that allocates nothing: the same kernels as rt_launch_flux_loss, with the
// partial sums in a static device array of RT_NOALLOC_PARTIALS + RT_BLOCK doubles (2 MiB).
#define RT_NOALLOC_PARTIALS ((1 << 18) - RT_BLOCK)
#define RT_MAX_DEVICES 64
int64_t rt_loss_blocks(int64_t N, int K);  // partial sums one loss launch writes
hipError_t rt_launch_flux_loss_noalloc(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light,
                                       const void *I, const double *face_weight, double *loss, void *seed, int dtype,
                                       hipStream_t s);
hipError_t rt_launch_moments(const rt_mesh *m, int K, const double *dirs, const double *W, double c_light,
                             const void *I, double *out, int dtype, int paired, hipStream_t s);
hipError_t rt_launch_diagnostics(const rt_mesh *m, int K, const double *dirs, const double *W, double c_red,
                                 double c_light, const void *I, const double *vol, const double *etot,
                                 const double *mom, double *out_dev, int dtype, hipStream_t s);

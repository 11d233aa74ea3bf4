// The radiation step kernel: transport (section 2.2) and the implicit source
// update (section 2.3) of one cell per group of LPC lanes, each lane holding APL
// angles.  One pass reads the cell's intensity row, gathers the neighbour rows of
// its faces through the half-face index (no atomics), updates the charges, runs the
// source on the transported row while it is in registers, and writes the row once.
#include "rt_source_vjp.h"
#include "rt_step_common.h"

namespace {

// Faces gathered per batch: all their neighbour-row loads are issued before any is
// used, so one memory round trip serves U faces.  At 128^3 x 80: two faces measured ~2%
// faster than four in FP32.  The FP64 form with antipodes side by side ran 5% faster with
// three (1.91 against 2.00 ms) at two waves per SIMD; since its source holds fewer values
// (three waves) two are faster again: 1.85 ms, against 2.45 ms with three.
template <typename T, int PAIRED> struct rt_batch {
  static constexpr int U = 2;
};

// MODE 0: source only (in place); 1: upwind transport (+ source); 2: reconstructed
// transport of PLM stage 2 (+ source); 3: the transpose of upwind transport (the
// adjoint: input mu = lam*/V' per cell and angle, output lam_i = V_i mu_i - sum over the
// faces the cell is upwind of, g > 0, of g (mu_i - mu_j)); 4: the transpose of step
// n + 1 followed, in registers, by the reverse of the source of step n (output lam*/V'
// of step n, so consecutive launches chain the reverse of a run of steps without
// storing dL/dI in between); 5: the reverse of the source of step n alone (input dL/dI
// of its output, read from the cell's own row only).  Separate instantiations keep each
// one's registers to what its own code needs.
//
// The cells of a workgroup are consecutive, so their half-faces form one contiguous
// range; it is staged in LDS (dynamic size: the largest range of any workgroup,
// found at upload) and the face loops read their records from there.
// Occupancy target: the FP64 PLM stage 2 (four rows gathered per face) would take all 256
// registers at one wave per SIMD; held to two it spills ~130 bytes per lane and runs 5%
// faster with antipodes K/2 apart (64^3 x 80 PLM step 1.96 -> 1.87 ms; unchanged with them
// side by side).  Everything else keeps the compiler's choice.
template <typename T, int MODE> struct rt_step_waves {
  static constexpr int value = MODE == 2 && sizeof(T) == 8 ? 2 : 1;
};
template <typename T, int LPC, int APL, int MODE, bool FULL, int PAIRED>
__global__ __launch_bounds__(RT_BLOCK) __attribute__((amdgpu_waves_per_eu(rt_step_waves<T, MODE>::value))) void
k_step(rt_step_args a, int64_t nblk) {
  using V4 = typename rt_vec4<T>::type;
  // Runs of two pairs per lane (fewer, wider gathers): at 128^3 x 80 upwind, FP32 with
  // antipodes side by side 1.30 -> 1.18 ms and FP64 with antipodes K/2 on 2.35 -> 2.04 ms
  // (the other two forms within 3%).  PLM stage 2 addresses its four gathered rows per
  // element and keeps one pair per slot (the runs made its FP64 form 1.59 -> 2.09 ms).
  using Ang = rt_step_angles<T, LPC, APL, FULL, PAIRED, MODE != 2>;
  constexpr bool FACES = MODE >= 1 && MODE <= 4;  // the modes that read face records
  constexpr bool TRANSPOSE = MODE == 3 || MODE == 4;
  constexpr int P = Ang::P;
  constexpr int U = rt_batch<T, PAIRED>::U;
  constexpr int CPB = RT_BLOCK / LPC;
  extern __shared__ __align__(16) unsigned char rt_smem[];
  V4 *s_an = (V4 *)rt_smem;
  V4 *s_rel = s_an + a.hf_cap;
  int32_t *s_nbr = (int32_t *)(s_an + (MODE == 2 ? 3 : 1) * a.hf_cap);
  const int64_t lb = rt_logical_block(nblk);
  if (lb < 0) return;  // whole padding workgroup
  const int64_t c0 = lb * CPB;
  const int g = threadIdx.x / LPC;
  const bool live = c0 + g < a.N;
  const int64_t cell = live ? c0 + a.wg_order[c0 + g] : c0;
  const int l = threadIdx.x % LPC;
  const int K = a.K;
  int H0 = 0;
  if (FACES) {
    const V4 *an = (const V4 *)a.hf_an;
    const V4 *rel = (const V4 *)a.hf_rel;
    const int64_t c1 = c0 + CPB < a.N ? c0 + CPB : a.N;
    H0 = a.row_ptr[c0];
    const int nH = a.row_ptr[c1] - H0;  // <= hf_cap by construction
    for (int i = threadIdx.x; i < nH; i += RT_BLOCK) {
      s_nbr[i] = a.hf_nbr[H0 + i];
      s_an[i] = an[H0 + i];
      if (MODE == 2) {
        s_rel[2 * i] = rel[2 * (H0 + i)];
        s_rel[2 * i + 1] = rel[2 * (H0 + i) + 1];
      }
    }
    __syncthreads();
  }
  if (!live) return;
  Ang ang;
  ang.load(a.dirs, a.W, K, l);

  const T *Iin = (const T *)a.I_in;
  const int64_t row = cell * (int64_t)K;
  // the lane's base pointers into row 0 (its first angle, and its lone pair's angle)
  const int k_single = Ang::SINGLE ? ang.k[P - 1] : ang.k[0];
  const T *Iin_lane = Iin + ang.k[0], *Iin_single = Iin + k_single;
  T Ic[APL];
  ang.read_lane(Iin_lane + row, Iin_single + row, Ic);

  double Vnew = 0.0, Vstart = 0.0;
  // the start-of-step volume: the reverse modes take it from the forward step's tape
  const double *tape = a.src_tape ? a.src_tape + RT_SRC_TAPE * cell : nullptr;
  const bool vol_from_tape = MODE >= 4 || (MODE == 3 && tape);
  if (MODE == 5) Vnew = rt_vol_next(tape[RT_TAPE_V], a.dt, a.D[cell]);
  if (FACES) {
    // ---- transport: charges V I minus the upwind charge through every face -------------
    const double Vn = vol_from_tape ? tape[RT_TAPE_V] : a.vol_in[cell];
    Vstart = Vn;
    const double dV = a.dt * a.D[cell];
    Vnew = rt_vol_next(Vn, a.dt, a.D[cell]);  // the end-of-step volume
    // the charge through the faces is accumulated apart from V I (the transpose adds V mu,
    // with V the start-of-step volume of the step it transposes: step n + 1 in mode 4)
    T acc[APL];
#pragma unroll
    for (int q = 0; q < APL; ++q) acc[q] = TRANSPOSE ? (T)(MODE == 4 ? Vnew : Vn) * Ic[q] : T(0);
    const T sc = (T)(a.dt * a.c_red), sd = (T)a.dt;
    const int h0 = a.row_ptr[cell], h1 = a.row_ptr[cell + 1];
    // a neighbour's row is one multiply-add away from the lane's base pointers
    const uint32_t row_bytes = (uint32_t)(K * sizeof(T));
    if (MODE == 1 || TRANSPOSE) {
      for (int h = h0; h < h1; h += U) {
        // batch metadata; slots past the cell's last face reuse face h0 with a zero record
        uint32_t j[U];
        V4 r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool v = h + u < h1;
          const int i = (v ? h + u : h0) - H0;
          j[u] = (uint32_t)s_nbr[i];
          r[u] = s_an[i];
          if (!v) r[u] = V4{T(0), T(0), T(0), T(0)};
        }
        T xn[U][APL];
#pragma unroll
        for (int u = 0; u < U; ++u)
          ang.read_lane(ang.lane_row(Iin_lane, j[u], row_bytes), ang.lane_row(Iin_single, j[u], row_bytes), xn[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // g = dt (cbar (A n_out).n_k - A (w~.n)_out): charge leaving per unit upwind intensity,
          // as three fused multiply-adds from -dt A (w~.n)_out.  Every operand of the face's
          // other side is negated exactly, so both sides get bitwise opposite g (conservation).
          const T ax = sc * r[u].x, ay = sc * r[u].y, az = sc * r[u].z, nb = -(sd * r[u].w);
          const T m2b = nb + nb;  // -2 dt A (w~.n)_out, exact
#pragma unroll
          for (int q = 0; q < P; ++q) {
            const T g = fma(az, ang.z[q], fma(ay, ang.y[q], fma(ax, ang.x[q], nb)));
            if constexpr (MODE == 1) {
              acc[q] -= g * (g > T(0) ? Ic[q] : xn[u][q]);
            } else {
              acc[q] -= g > T(0) ? g * (Ic[q] - xn[u][q]) : T(0);
            }
            if (PAIRED) {
              const T g2 = m2b - g;  // the antipodal angle: -(dot) - b
              if constexpr (MODE == 1) {
                acc[q + P] -= g2 * (g2 > T(0) ? Ic[q + P] : xn[u][q + P]);
              } else {
                acc[q + P] -= g2 > T(0) ? g2 * (Ic[q + P] - xn[u][q + P]) : T(0);
              }
            }
          }
        }
      }
    } else {
      // reconstructed face states of the half-step intensities (PLM stage 2).  FP32: each cell
      // and angle's (I_half, limited gradient) is one 16-byte 4-vector ([N][K][4]), so a face
      // state is one access (64^3 x 80 PLM step 0.94 -> 0.85 ms); FP64 keeps I_half [N][K] and
      // the gradient [N][3][K] apart (packed, its 32-byte states raised the register pressure
      // of a kernel already spilling: 1.57 -> 2.07 ms)
      constexpr bool PACKED = sizeof(T) == 4;
      const V4 *Pk = (const V4 *)a.grad;
      const T *Ih = (const T *)a.I_half;
      const T *G = (const T *)a.grad;
      T hs[APL], gsx[APL], gsy[APL], gsz[APL];
#pragma unroll
      for (int q = 0; q < APL; ++q) {
        const int k = ang.k[q];
        if constexpr (PACKED) {
          const V4 o = Pk[row + k];
          hs[q] = o.x;
          gsx[q] = o.y;
          gsy[q] = o.z;
          gsz[q] = o.w;
        } else {
          hs[q] = Ih[row + k];
          gsx[q] = G[(cell * 3 + 0) * K + k];
          gsy[q] = G[(cell * 3 + 1) * K + k];
          gsz[q] = G[(cell * 3 + 2) * K + k];
        }
      }
      constexpr int UP = sizeof(T) == 4 ? 2 : 1;
      for (int h = h0; h < h1; h += UP) {
        uint32_t j[UP];
        V4 r[UP], r0[UP], r1[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          const bool v = h + u < h1;
          const int i = (v ? h + u : h0) - H0;
          j[u] = (uint32_t)s_nbr[i];
          r[u] = s_an[i];
          r0[u] = s_rel[2 * i];
          r1[u] = s_rel[2 * i + 1];
          if (!v) r[u] = V4{T(0), T(0), T(0), T(0)};
        }
        T xh[UP][APL], xg0[UP][APL], xg1[UP][APL], xg2[UP][APL];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          if constexpr (PACKED) {
            const V4 *Pj = Pk + (uint64_t)j[u] * K;
#pragma unroll
            for (int q = 0; q < APL; ++q) {
              const V4 o = Pj[ang.k[q]];
              xh[u][q] = o.x;
              xg0[u][q] = o.y;
              xg1[u][q] = o.z;
              xg2[u][q] = o.w;
            }
          } else {
            const T *Hj = Ih + (uint64_t)j[u] * K;
            const T *Gj = G + (uint64_t)j[u] * 3 * K;
#pragma unroll
            for (int q = 0; q < APL; ++q) {
              const int k = ang.k[q];
              xh[u][q] = Hj[k];
              xg0[u][q] = Gj[k];
              xg1[u][q] = Gj[K + k];
              xg2[u][q] = Gj[2 * K + k];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          const T ax = sc * r[u].x, ay = sc * r[u].y, az = sc * r[u].z, nb = -(sd * r[u].w);
          const T m2b = nb + nb;
          // the charge through the face at the reconstructed state of its upwind side
          auto face = [&](int q, T g) {
            const T fs = hs[q] + gsx[q] * r0[u].x + gsy[q] * r0[u].y + gsz[q] * r0[u].z;
            const T fn = xh[u][q] + xg0[u][q] * r0[u].w + xg1[u][q] * r1[u].x + xg2[u][q] * r1[u].y;
            acc[q] -= g * (g > T(0) ? fs : fn);
          };
          // FP32: the antipode's speed as in the upwind loop (64^3 x 80 PLM step 0.778 ->
          // 0.760 ms); FP64 keeps three multiply-adds per angle (paired: 1.474 -> 1.489 ms)
          constexpr bool PAIR_G = PAIRED && sizeof(T) == 4;
          constexpr int NG = PAIR_G ? P : APL;
#pragma unroll
          for (int q = 0; q < NG; ++q) {
            const T g = fma(az, ang.dz(q), fma(ay, ang.dy(q), fma(ax, ang.dx(q), nb)));
            face(q, g);
            if (PAIR_G) face(q + P, m2b - g);
          }
        }
      }
    }
    if constexpr (TRANSPOSE) {
#pragma unroll
      for (int q = 0; q < APL; ++q) Ic[q] = acc[q];
    } else {
      // I' = I (V/V') + (charge through the faces)/V'.  The ratio V/V' = 1 - dt D/V' is
      // formed in FP64, so on a still mesh it is exactly one: the stored intensities then
      // carry no per-cell rounding of V that would repeat, with one sign, every step.
      const double iV = rt_rcp(Vnew);
      const T cr = (T)(1.0 - dV * iV), ci = (T)iV;
#pragma unroll
      for (int q = 0; q < APL; ++q) Ic[q] = Ic[q] * cr + acc[q] * ci;
    }
    if constexpr (MODE == 1) {
      if (a.I_star_out) {
        T *o = (T *)a.I_star_out + row;
        ang.write_lane(o + ang.k[0], o + k_single, Ic);
      }
    }
  }

  if constexpr (MODE <= 2) {
    if (a.do_source) rt_source_cell<T, LPC, APL>(a, ang, cell, l, Ic);
  }
  if constexpr (MODE >= 4) {
    // Ic holds dL/dI^{n+1} of the cell; the reverse of the source of step n turns it into
    // dL/dI* / V' (V' = Vnew, the end-of-step volume of step n), reading the step's output
    T Io[APL];
    const T *In = (const T *)a.I_next + row;
    ang.read_lane(In + ang.k[0], In + k_single, Io);
    rt_source_vjp_cell<T, LPC, APL>(a, ang, cell, l, Io, Ic, Vnew);
  }

  {
    T *o = (T *)a.I_out + row;
    ang.write_lane(o + ang.k[0], o + k_single, Ic);
  }
  if ((MODE == 1 || MODE == 2) && l == 0 && a.vol_out) a.vol_out[cell] = Vnew;
  if (MODE == 1 && l == 0 && a.src_tape_out) a.src_tape_out[RT_SRC_TAPE * cell + RT_TAPE_V] = Vstart;
}

// Staging needs (records per half-face) x (half-faces of the largest range of the
// workgroup's cells) bytes of LDS; a layout that would need more than a workgroup may
// use (160 KiB on gfx950) is refused with hipErrorInvalidConfiguration (the dispatch then
// tries the general layout, whose 16-cell workgroups the upload checked to fit).
template <typename T, int LPC, int APL, bool FULL, int PAIRED>
hipError_t launch_mode(const rt_step_args &args, hipStream_t s) {
  using V4 = typename rt_vec4<T>::type;
  rt_step_args a = args;
  a.hf_cap = LPC == 16 ? a.hf_cap16 : LPC == 8 ? a.hf_cap32 : a.hf_cap64;
  a.wg_order = LPC == 16 ? a.wg_order16 : LPC == 8 ? a.wg_order32 : a.wg_order64;
  const int64_t cpb = RT_BLOCK / LPC;
  const int64_t nblk = (a.N + cpb - 1) / cpb;
  const dim3 grid((unsigned)rt_grid_for(nblk)), block(RT_BLOCK);
  const size_t per = (a.do_transport == 2 ? 3 : 1) * sizeof(V4) + sizeof(int32_t);
  const bool faces = a.do_transport >= 1 && a.do_transport <= 4;
  const size_t smem = faces ? per * (size_t)a.hf_cap : 0;
  if (smem > (size_t)a.lds_max) return hipErrorInvalidConfiguration;
  switch (a.do_transport) {
    case 0: hipLaunchKernelGGL((k_step<T, LPC, APL, 0, FULL, PAIRED>), grid, block, smem, s, a, nblk); break;
    case 1: hipLaunchKernelGGL((k_step<T, LPC, APL, 1, FULL, PAIRED>), grid, block, smem, s, a, nblk); break;
    case 2: hipLaunchKernelGGL((k_step<T, LPC, APL, 2, FULL, PAIRED>), grid, block, smem, s, a, nblk); break;
    case 3: hipLaunchKernelGGL((k_step<T, LPC, APL, 3, FULL, PAIRED>), grid, block, smem, s, a, nblk); break;
    case 4: hipLaunchKernelGGL((k_step<T, LPC, APL, 4, FULL, PAIRED>), grid, block, smem, s, a, nblk); break;
    case 5: hipLaunchKernelGGL((k_step<T, LPC, APL, 5, FULL, PAIRED>), grid, block, smem, s, a, nblk); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int LPC, int APL> hipError_t launch(const rt_step_args &a, hipStream_t s) {
  return a.K == LPC * APL ? launch_mode<T, LPC, APL, true, 0>(a, s)
                          : launch_mode<T, LPC, APL, false, 0>(a, s);
}

template <typename T, int PAIRED> hipError_t dispatch_paired(const rt_step_args &a, hipStream_t s) {
  switch (rt_paired_lanes(a.K)) {  // 0 (no paired layout for K) matches no case
    case 0x0802: return launch_mode<T, 8, 2, true, PAIRED>(a, s);
    case 0x0804: return launch_mode<T, 8, 4, true, PAIRED>(a, s);
    case 0x0806: return launch_mode<T, 8, 6, true, PAIRED>(a, s);
    case 0x0808: return launch_mode<T, 8, 8, true, PAIRED>(a, s);
    case 0x080a: return launch_mode<T, 8, 10, true, PAIRED>(a, s);
    case 0x080c: return launch_mode<T, 8, 12, true, PAIRED>(a, s);
    case 0x0402: return launch_mode<T, 4, 2, true, PAIRED>(a, s);
    case 0x0406: return launch_mode<T, 4, 6, true, PAIRED>(a, s);
    case 0x040a: return launch_mode<T, 4, 10, true, PAIRED>(a, s);
  }
  return hipErrorInvalidConfiguration;
}

template <typename T> hipError_t dispatch_general16(const rt_step_args &a, hipStream_t s) {
  switch ((a.K + 15) / 16) {
    case 1: return launch<T, 16, 1>(a, s);
    case 2: return launch<T, 16, 2>(a, s);
    case 3: return launch<T, 16, 3>(a, s);
    case 4: return launch<T, 16, 4>(a, s);
    case 5: return launch<T, 16, 5>(a, s);
    case 6: return launch<T, 16, 6>(a, s);
    case 7: return launch<T, 16, 7>(a, s);
    case 8: return launch<T, 16, 8>(a, s);
  }
  return hipErrorInvalidValue;
}

// The general layout for K; when 8 lanes per cell (32-cell workgroups) cannot stage their
// face records, 16 lanes (16-cell workgroups, which the upload checked to fit) serve K.
template <typename T> hipError_t dispatch_general(const rt_step_args &a, hipStream_t s) {
  const int lanes = rt_step_lanes(a.K, 0);
  if ((lanes >> 8) == 16) return dispatch_general16<T>(a, s);
  hipError_t e = hipErrorInvalidValue;
  switch (lanes) {
    case 0x0801: e = launch<T, 8, 1>(a, s); break;
    case 0x0802: e = launch<T, 8, 2>(a, s); break;
    case 0x0803: e = launch<T, 8, 3>(a, s); break;
    case 0x0804: e = launch<T, 8, 4>(a, s); break;
    case 0x0805: e = launch<T, 8, 5>(a, s); break;
    case 0x0806: e = launch<T, 8, 6>(a, s); break;
    case 0x0807: e = launch<T, 8, 7>(a, s); break;
    case 0x0808: e = launch<T, 8, 8>(a, s); break;
  }
  return e == hipErrorInvalidConfiguration ? dispatch_general16<T>(a, s) : e;
}

// Antipodal sets take the paired kernel when it has a lane layout for K and its staging
// fits in LDS; everything else (and that fallback) the general kernel.
template <typename T> hipError_t dispatch(const rt_step_args &a, hipStream_t s) {
  if (a.paired) {
    const hipError_t e = a.paired == 2 ? dispatch_paired<T, 2>(a, s) : dispatch_paired<T, 1>(a, s);
    if (e != hipErrorInvalidConfiguration) return e;
  }
  return dispatch_general<T>(a, s);
}

}  // namespace

hipError_t rt_launch_step(const rt_step_args &a, int dtype, hipStream_t s) {
  return dtype == RT_F32 ? dispatch<float>(a, s) : dispatch<double>(a, s);
}

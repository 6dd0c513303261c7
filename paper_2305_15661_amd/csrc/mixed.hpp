// Mixed-precision EQ assembly: point physics in FP32 (Pts<D, float>), the
// projection M_e = sqrt(rho_e) [Aw Bw | Ax Bx] on BF16 matrix cores with FP32
// accumulation, and the Gram reduction M_e^T M_e, the gradient and the
// objective accumulated in FP64 (as the FP64 path does).
//
// The contraction index is re-blocked so that each 16-wide k-step of the
// 16x16x16 BF16 MFMA lies inside one region (volume / face minus / face
// plus for Aw; volume / face for Ax); regions are zero-padded to multiples
// of 16.  Lane l of a k-step supplies A[l%16][4 (l/16) + t] and
// B[4 (l/16) + t][l%16], t < 4, and accumulator register v holds row
// 4 (l/16) + v of column l%16.  Register v of a projection tile therefore
// holds rows {v, 4 + v, 8 + v, 12 + v}: a k-block of the FP64 16x16x4 MFMA
// in exactly its operand layout, so the Gram uses the FP32 accumulators
// (widened) without moving data.
#pragma once
#include "batch.hpp"

namespace ift {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));

template <class D>
struct EqOp16 {
  static constexpr int KV = D::NQV * D::NC;
  static constexpr int KF = 3 * D::NQF * D::NC;
  static constexpr int KV16 = (KV + 15) / 16 * 16;
  static constexpr int KF16 = (KF + 15) / 16 * 16;
  static constexpr int KW16 = KV16 + 2 * KF16;
  static constexpr int KXV = 4 * D::NQV;
  static constexpr int KXF = EqOp<D>::KXF + EqOp<D>::KXQ;   // face rows, then Burgers source-position rows
  static constexpr int KXV16 = (KXV + 15) / 16 * 16;
  static constexpr int KXF16 = (KXF + 15) / 16 * 16;
  static constexpr int KX16 = KXV16 + KXF16;
};

IFT_DEV short to_bf16(float x) { return __builtin_bit_cast(short, (__bf16)x); }

// Original row of Bw (EqOp order) for re-blocked index kk, or -1 (padding).
template <class D>
IFT_DEV int w16_row(int kk) {
  using O = EqOp16<D>;
  if (kk < O::KV16) return kk < O::KV ? kk : -1;
  const int r = kk - O::KV16;
  const int plus = r >= O::KF16;
  const int cf = r - (plus ? O::KF16 : 0);
  return cf < O::KF ? O::KV + plus * O::KF + cf : -1;
}

template <class D>
IFT_DEV int x16_row(int kk) {
  using O = EqOp16<D>;
  if (kk < O::KXV16) return kk < O::KXV ? kk : -1;
  const int cf = kk - O::KXV16;
  return cf < O::KXF ? O::KXV + cf : -1;
}

// BF16 point bases, column-major per element so that a lane's four k-entries
// of one column are one 8-byte load:  Bw16 [n_s][n + 1][KW16],
// Bx16 [n_s][m + 1][KX16] (last column and padded k-entries zero), from the
// FP64 bases Bw [n_s][KWP][n + 1] and Bx [n_s][KXP][m + 1].
template <class D>
__global__ __launch_bounds__(256) void k_point_bases16(const double* Bw, const double* Bx, int n, int m, short* Bw16,
                                                       short* Bx16) {
  using O = EqOp<D>;
  using Q = EqOp16<D>;
  const int k = blockIdx.x;
  const int lw = n + 1, lx = m + 1;
  for (int e = threadIdx.x; e < lw * Q::KW16; e += 256) {
    const int j = e / Q::KW16, kk = e % Q::KW16;
    const int r = w16_row<D>(kk);
    const double v = r >= 0 ? Bw[((long long)k * O::KWP + r) * lw + j] : 0.0;
    Bw16[(long long)k * lw * Q::KW16 + e] = to_bf16(float(v));
  }
  for (int e = threadIdx.x; e < lx * Q::KX16; e += 256) {
    const int j = e / Q::KX16, kk = e % Q::KX16;
    const int r = x16_row<D>(kk);
    const double v = r >= 0 ? Bx[((long long)k * O::KXP + r) * lx + j] : 0.0;
    Bx16[(long long)k * lx * Q::KX16 + e] = to_bf16(float(v));
  }
}

// The four A entries (row r, re-blocked columns 4 kq + t) of a w k-step in
// region `reg` (0 volume, 1 face minus, 2 face plus), FP32, branch-free.
template <class D>
IFT_DEV void aw16(const RefTab& t, const Pts<D, float>& p, int i, int c, float rm, int reg, int c0, float* out) {
  using Q = EqOp16<D>;
  constexpr int NC = D::NC;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int col = c0 + u;   // column inside the region
    float v;
    if (reg == 0) {
      const float ok = col < Q::KV ? 1.f : 0.f;
      const int cc0 = col < Q::KV ? col : 0;
      const int q = cc0 / NC, cc = cc0 % NC;
      v = -float(t.wv[q]) * (p.gp[q][i][0] * p.Af[q][c][0][cc] + p.gp[q][i][1] * p.Af[q][c][1][cc]) * ok;
    } else {
      const float ok = col < Q::KF ? 1.f : 0.f;
      const int cf = col < Q::KF ? col : 0;
      const int f = cf / (D::NQF * NC), q = (cf / NC) % D::NQF, cc = cf % NC;
      const float hp = p.dHp[f][q][c][cc], hm = p.dHm[f][q][c][cc];
      const float sp = reg == 2 ? 1.f : 0.f;
      v = float(t.wl[i][f][q]) * (hp * sp + hm * (1.f - sp)) * ok;
    }
    out[u] = v * rm;
  }
}

template <class D>
IFT_DEV void ax16(const RefTab& t, const Pts<D, float>& p, int i, int c, float rm, int reg, int c0, float* out) {
  using Q = EqOp16<D>;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int col = c0 + u;
    float v;
    if (reg == 0) {
      const float ok = col < Q::KXV ? 1.f : 0.f;
      const int cv = col < Q::KXV ? col : 0;
      const int q = cv >> 2, ab = cv & 3;
      const float px = float(t.dphiv[q][i][0]), py = float(t.dphiv[q][i][1]);
      const float f0 = p.fv[q][c][0], f1 = p.fv[q][c][1];
      const float s1 = ab < 2 ? 1.f : 0.f, s2 = (ab & 1) ? 1.f : 0.f;
      const float sg = (ab == 0 || ab == 3) ? -1.f : 1.f;
      v = sg * float(t.wv[q]) * (f1 * s1 + f0 * (1.f - s1)) * (px * s2 + py * (1.f - s2));
      if constexpr (D::PDE == PDE_BURGERS) v -= float(t.wv[q] * t.phiv[q][i]) * p.src[q][1 + ab];
      v *= ok;
    } else {
      const float ok = col < Q::KXF ? 1.f : 0.f;
      const int cf0 = col < Q::KXF ? col : 0;
      constexpr int NF = EqOp<D>::KXF;
      const int cf = cf0 < NF ? cf0 : 0;
      const int f = cf / (2 * D::NQF), q = (cf >> 1) % D::NQF, d = cf & 1;
      const float h0 = p.dHn[f][q][c][0], h1 = p.dHn[f][q][c][1];
      const float sd = d == 0 ? 1.f : 0.f;
      v = float(t.wl[i][f][q]) * (-h1 * sd + h0 * (1.f - sd));
      if constexpr (EqOp<D>::KXQ > 0) {
        // source-position row qq: -w_q phi_i b det J s_q
        const int qq = cf0 >= NF ? cf0 - NF : 0;
        const float vq = -float(t.wv[qq] * t.phiv[qq][i]) * p.src[qq][5];
        const float sf = cf0 < NF ? 1.f : 0.f;
        v = v * sf + vq * (1.f - sf);
      }
      v *= ok;
    }
    out[u] = v * rm;
  }
}

// One block of the mixed fused assembly (same contract as fused_body).
template <class D, int NT>
IFT_DEV void fused_body_mixed(FusedShared<D, float, NT>& sh, const EqArgs& a, const short* Bw16, const short* Bx16,
                              const FusedArgs& f, int blk, int pt) {
  using Q = EqOp16<D>;
  constexpr int NUE = D::NUE;
  constexpr int MT = (NUE + 1 + 15) / 16;
  constexpr int NH = NT * (NT + 1) / 2;
  // distortion row nue: tile NUE / 16, lane group kq and register v with 4 kq + v = NUE % 16
  constexpr int RD_MT = NUE / 16, RD_K = (NUE % 16) / 4, RD_V = (NUE % 16) % 4;
  const RefTab& tab = sh.tab;
  auto& u = sh.u;
  auto& sbad = sh.sbad;
  const int n = a.n, m = a.m, Dd = a.D;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int kq = lane >> 4, li = lane & 15;
  dvec4 h[NH];
#pragma unroll
  for (int t = 0; t < NH; ++t) h[t] = dvec4{0.0, 0.0, 0.0, 0.0};
  int nbad = 0, bor = 0;
  const long long nrow_e = (long long)a.n_s * NUE;
  const long long po = (long long)pt * a.nrows;
  const int kbeg = (blk * (NTHR / 64) + wave) * f.E;
  FusedSlot<D, float>& S = u.w[wave][0];
  for (int e = 0; e < f.E; ++e) {
    const int k = kbeg + e;
    __syncthreads();
    if (k < a.n_s) copy_pts_wave<D, float>(&S.p, reinterpret_cast<const Pts<D, float>*>(a.pts) + ((long long)pt * a.n_s + k), lane);
    __syncthreads();
    if (k >= a.n_s) continue;
    const Pts<D, float>& p = S.p;
    const float sq = float(a.srho[k]);
    float rv = 0.f;
    if (lane < NUE) rv = residual_entry_p<D, float>(p, tab, lane);
    else if (lane == NUE) rv = p.N;
    const float dv = lane < m ? p.dv[lane] : 0.f;   // distortion row entry of x-column `lane`
    f32x4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    int ri[MT], rc[MT];
    float rm[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = 16 * mt + li;
      rm[mt] = row < NUE ? 1.f : 0.f;
      ri[mt] = (row < NUE ? row : 0) / D::NC;
      rc[mt] = (row < NUE ? row : 0) % D::NC;
    }
    // B: column c of this lane (zero column past the block), k-entries 4 kq .. 4 kq + 3
    const short* bw = Bw16 + (long long)k * (n + 1) * Q::KW16;
    const short* bx = Bx16 + (long long)k * (m + 1) * Q::KX16;
    int cw[NT], cx[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int c = 16 * nt + li, jx = c - n;
      cw[nt] = c < n ? c : n;
      cx[nt] = (jx >= 0 && jx < m) ? jx : m;
    }
#pragma unroll 1
    for (int s = 0; s < Q::KW16 / 16; ++s) {
      const int reg = 16 * s < Q::KV16 ? 0 : (16 * s < Q::KV16 + Q::KF16 ? 1 : 2);
      const int c0 = 16 * s - (reg == 0 ? 0 : (reg == 1 ? Q::KV16 : Q::KV16 + Q::KF16)) + 4 * kq;
      bf16x4 bv[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        bv[nt] = *reinterpret_cast<const bf16x4*>(bw + (long long)cw[nt] * Q::KW16 + 16 * s + 4 * kq);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        float av[4];
        aw16<D>(tab, p, ri[mt], rc[mt], rm[mt], reg, c0, av);
        bf16x4 ab;
#pragma unroll
        for (int t = 0; t < 4; ++t) ab[t] = to_bf16(av[t]);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ab, bv[nt], acc[mt][nt], 0, 0, 0);
      }
    }
    if (m > 0) {
#pragma unroll 1
      for (int s = 0; s < Q::KX16 / 16; ++s) {
        const int reg = 16 * s < Q::KXV16 ? 0 : 1;
        const int c0 = 16 * s - (reg == 0 ? 0 : Q::KXV16) + 4 * kq;
        bf16x4 bv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          bv[nt] = *reinterpret_cast<const bf16x4*>(bx + (long long)cx[nt] * Q::KX16 + 16 * s + 4 * kq);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          float av[4];
          ax16<D>(tab, p, ri[mt], rc[mt], rm[mt], reg, c0, av);
          bf16x4 ab;
#pragma unroll
          for (int t = 0; t < 4; ++t) ab[t] = to_bf16(av[t]);
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ab, bv[nt], acc[mt][nt], 0, 0, 0);
        }
      }
    }
    // scale; residual column and distortion row (register v of lane group
    // kq holds row 4 kq + v)
    float dsrc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int jd = 16 * nt + li - n;
      dsrc[nt] = __shfl(dv, (jd >= 0 && jd < 64) ? jd : 0);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * mt + 4 * kq + v;   // < 32
        const float rsrc = __shfl(rv, row);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int c = 16 * nt + li, jd = c - n;
          float x = sq * acc[mt][nt][v];
          if (c == Dd) x = sq * rsrc;
          else if (mt == RD_MT && kq == RD_K && v == RD_V && jd >= 0 && jd < m) x = sq * dsrc[nt];
          acc[mt][nt][v] = x;
        }
      }
    if (f.rows) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * mt + 4 * kq + v, c = 16 * nt + li;
            if (row > NUE || c > Dd) continue;
            const long long gr = row < NUE ? (long long)k * NUE + row : nrow_e + k;
            if (c < Dd) a.Jt[(po + gr) * Dd + c] = double(acc[mt][nt][v]);
            else a.Ft[po + gr] = double(acc[mt][nt][v]);
          }
    }
    // Gram in FP64: register v of every row tile is one k-block
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (16 * mt + v > NUE) continue;
        int t = 0;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
          for (int tb = ta; tb < NT; ++tb, ++t)
            h[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(double(acc[mt][ta][v]), double(acc[mt][tb][v]), h[t], 0, 0, 0);
      }
    const int bad = p.bad;
    nbad += bad != 0;
    bor |= bad;
    if (f.rows && lane == 0) a.flags[(long long)pt * a.n_s + k] = bad;
  }
  __syncthreads();
  if (lane == 0) {
    sbad[wave][0] = nbad;
    sbad[wave][1] = bor;
  }
  double* part = f.part + ((long long)pt * f.nblk + blk) * NH * 256;
#pragma unroll
  for (int t = 0; t < NH; ++t) {
    if (wave > 0)
#pragma unroll
      for (int v = 0; v < 4; ++v) u.red[wave - 1][v * 64 + lane] = h[t][v];
    __syncthreads();
    if (wave == 0)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double x = h[t][v];
#pragma unroll
        for (int w = 0; w < NTHR / 64 - 1; ++w) x += u.red[w][v * 64 + lane];
        part[t * 256 + v * 64 + lane] = x;
      }
    __syncthreads();
  }
  if (tid == 0) {
    int c = 0, o = 0;
    for (int w = 0; w < NTHR / 64; ++w) {
      c += sbad[w][0];
      o |= sbad[w][1];
    }
    f.part_bad[((long long)pt * f.nblk + blk) * 2] = c;
    f.part_bad[((long long)pt * f.nblk + blk) * 2 + 1] = o;
  }
}

template <class D, int NT>
__global__ __launch_bounds__(NTHR) void k_eq_fused_mixed(EqArgs a, const short* Bw16, const short* Bx16, FusedArgs f) {
  __shared__ FusedShared<D, float, NT> sh;
  fused_load_tab<D, float, NT>(sh, threadIdx.x);
  fused_body_mixed<D, NT>(sh, a, Bw16, Bx16, f, blockIdx.x, blockIdx.y);
}

// As k_fused_batch, for the instances in their mixed-precision rounds.
template <class D, int NT>
__global__ __launch_bounds__(NTHR) void k_fused_batch_mixed(const BatchInst* I, BatchLists L, int n_inst, int E) {
  __shared__ FusedShared<D, float, NT> sh;
  fused_load_tab<D, float, NT>(sh, threadIdx.x);
  const int* off = L.off + NT * (n_inst + 1);
  const int total = L.cnt[NT];
  int inst = 0;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    inst = __builtin_amdgcn_readfirstlane(batch_owner_from(off, n_inst, item, inst));
    const int blk = item - off[inst];
    const BatchInst& bi = I[inst];
    FusedArgs f;
    f.E = E;
    f.nblk = bi.nblk;
    f.part = bi.part;
    f.part_bad = bi.part_bad;
    f.rows = 0;
    fused_body_mixed<D, NT>(sh, bi.a, bi.Bw16, bi.Bx16, f, blk, 0);
  }
}

}  // namespace ift

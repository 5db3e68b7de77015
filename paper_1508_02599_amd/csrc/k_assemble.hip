// Element assembly, local gathers, right-hand sides, rigid-body kernels and
// the coarse matrix G^T G.
//
// Element tangents: one wavefront per Q1 element, lane (a, b) computes the
// 3x3 block K_ab over the 2x2x2 Gauss points; one workgroup per Q2 element
// (3x3x3 Gauss points, below).
//   * isotropic linear elasticity (section 5.1);
//   * Holzapfel-Gasser-Ogden (section 2: eqs. (isoaniso), (iso), (aniso_1),
//     (aniso_2), stress split of eq. (additiveStress)) with the tangent of
//     eq. (Tangent) and a pressure that is constant per element and condensed
//     (section 3.2, P0 static condensation): mean dilatation Jbar = v_e/V_e,
//     p = kappa (Jbar - 1), plus the rank-one term (kappa/V_e) g g^T.
// The elasticity tensor, which the paper leaves to its references, is the
// closed form of the HGO energy: C = C_iso + C_vol with
//   C_iso = P:Cbar:P^T + 2/3 J^{-2/3} (Sbar:C) Ptilde - 2/3 (Cinv x S_iso + S_iso x Cinv),
//   C_vol = J p (Cinv x Cinv - 2 Cinv (.) Cinv).
// Gathers into the subdomain matrices sum the element blocks of every node pair
// in a fixed order (no atomics), so assembly is deterministic.
#include "feti_impl.h"
#include "k_pcg.h"

namespace feti {

__device__ __forceinline__ int64_t tidx3(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }

__device__ __forceinline__ double corner(int a, int k) { return (double)(2 * ((a >> k) & 1) - 1); }

// dN_a/dxi_k at Gauss point gp (points at +-1/sqrt(3), ordered like the corners)
__device__ __forceinline__ double dshape(int a, int k, int gp) {
  const double g = 0.57735026918962576451;
  double v = 0.125 * corner(a, k);
  for (int d = 0; d < 3; ++d)
    if (d != k) v *= 1.0 + corner(a, d) * corner(gp, d) * g;
  return v;
}
__device__ __forceinline__ double shape(int a, int gp) {
  const double g = 0.57735026918962576451;
  double v = 0.125;
  for (int d = 0; d < 3; ++d) v *= 1.0 + corner(a, d) * corner(gp, d) * g;
  return v;
}

// 1D quadratic Lagrange polynomial of node i (at -1, 0, 1) and its derivative.
__device__ __forceinline__ double lag3(int i, double x) {
  return i == 0 ? 0.5 * x * (x - 1.0) : (i == 1 ? 1.0 - x * x : 0.5 * x * (x + 1.0));
}
__device__ __forceinline__ double dlag3(int i, double x) { return i == 0 ? x - 0.5 : (i == 1 ? -2.0 * x : x + 0.5); }
// 3-point Gauss-Legendre rule on [-1, 1]: points 0, +-sqrt(3/5), weights 8/9, 5/9
constexpr double kG3 = 0.77459666924148337704;
__device__ __forceinline__ double gp3(int g) { return g == 0 ? -kG3 : (g == 1 ? 0.0 : kG3); }
__device__ __forceinline__ double gw3(int g) { return g == 1 ? 8.0 / 9.0 : 5.0 / 9.0; }

__device__ void inv3(const double* A, double* inv, double* det) {
  const double c00 = A[4] * A[8] - A[5] * A[7];
  const double c01 = -(A[3] * A[8] - A[5] * A[6]);
  const double c02 = A[3] * A[7] - A[4] * A[6];
  const double d = A[0] * c00 + A[1] * c01 + A[2] * c02;
  const double id = 1.0 / d;
  inv[0] = c00 * id;
  inv[3] = c01 * id;
  inv[6] = c02 * id;
  inv[1] = -(A[1] * A[8] - A[2] * A[7]) * id;
  inv[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  inv[7] = -(A[0] * A[7] - A[1] * A[6]) * id;
  inv[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  inv[5] = -(A[0] * A[5] - A[2] * A[3]) * id;
  inv[8] = (A[0] * A[4] - A[1] * A[3]) * id;
  *det = d;
}

__constant__ int VA[6] = {0, 1, 2, 0, 1, 0};
__constant__ int VB[6] = {0, 1, 2, 1, 2, 2};

// Per-Gauss-point HGO state: total S (sym 3x3), Voigt tangent, F.
struct HgoPoint {
  double S[9], CV[36], F[9];
};

// Closed-form isochoric + volumetric stress/tangent of the HGO model at C,
// with the element pressure p (P0) and the element factor J of this point.
__device__ __forceinline__ void hgo_point(const double* F, double J, double p, const double* a1, const double* a2, double c,
                          double k1, double k2, HgoPoint& out) {
  double C[9];
  for (int I = 0; I < 3; ++I)
    for (int K = 0; K < 3; ++K) C[3 * I + K] = F[I] * F[K] + F[3 + I] * F[3 + K] + F[6 + I] * F[6 + K];
  double Ci[9], detC;
  inv3(C, Ci, &detC);
  const double Jm23 = pow(J, -2.0 / 3.0);
  const double* af[2] = {a1, a2};
  double d1[2], d2[2], A[2][9], D[2][9];
  for (int f = 0; f < 2; ++f) {
    const double* a = af[f];
    double aCa = 0.0, aCIa = 0.0;
    for (int I = 0; I < 3; ++I)
      for (int K = 0; K < 3; ++K) {
        aCa += a[I] * C[3 * I + K] * a[K];
        aCIa += a[I] * (C[3 * I + K] - (I == K ? 1.0 : 0.0)) * a[K];
      }
    // Ibar_4 - 1 for a unit fibre, exactly zero at C = I
    const double E = Jm23 * aCIa + (Jm23 - 1.0);
    if (E > 0.0) {   // fibres carry tension only
      const double ex = exp(k2 * E * E);
      d1[f] = k1 * E * ex;
      d2[f] = k1 * (1.0 + 2.0 * k2 * E * E) * ex;
    } else {
      d1[f] = 0.0;
      d2[f] = 0.0;
    }
    for (int I = 0; I < 3; ++I)
      for (int K = 0; K < 3; ++K) A[f][3 * I + K] = a[I] * a[K];
    for (int k = 0; k < 9; ++k) D[f][k] = A[f][k] - aCa / 3.0 * Ci[k];   // dev_C(A)
  }
  double Sb[9];
  for (int k = 0; k < 9; ++k) Sb[k] = 2.0 * d1[0] * A[0][k] + 2.0 * d1[1] * A[1][k];
  Sb[0] += c;
  Sb[4] += c;
  Sb[8] += c;
  double SbC = 0.0;
  for (int k = 0; k < 9; ++k) SbC += Sb[k] * C[k];
  double Siso[9];
  for (int k = 0; k < 9; ++k) Siso[k] = Jm23 * (Sb[k] - SbC / 3.0 * Ci[k]);
  for (int k = 0; k < 9; ++k) {
    out.S[k] = Siso[k] + J * p * Ci[k];
    out.F[k] = F[k];
  }
  const double cbar0 = 4.0 * Jm23 * Jm23 * d2[0], cbar1 = 4.0 * Jm23 * Jm23 * d2[1];
  const double tr23 = 2.0 / 3.0 * Jm23 * SbC;
  for (int al = 0; al < 6; ++al) {
    const int a = VA[al], b = VB[al];
    for (int be = 0; be < 6; ++be) {
      const int cc = VA[be], d = VB[be];
      const double odot = 0.5 * (Ci[3 * a + cc] * Ci[3 * b + d] + Ci[3 * a + d] * Ci[3 * b + cc]);
      const double oxo = Ci[3 * a + b] * Ci[3 * cc + d];
      double v = cbar0 * D[0][3 * a + b] * D[0][3 * cc + d] + cbar1 * D[1][3 * a + b] * D[1][3 * cc + d];
      v += tr23 * (odot - oxo / 3.0);
      v -= 2.0 / 3.0 * (Ci[3 * a + b] * Siso[3 * cc + d] + Siso[3 * a + b] * Ci[3 * cc + d]);
      v += J * p * (oxo - 2.0 * odot);
      out.CV[6 * al + be] = v;
    }
  }
}

// One wavefront per element; 4 elements per 256-thread block.  Barriers are
// block-wide and unconditional; per-wave work is guarded by its element's kind.
__global__ __launch_bounds__(256) void k_elements(AsmArgs A) {
  __shared__ double sX[4][24], sU[4][24], sInv[4][8][9], sDet[4][8], sdN[4][8][8][3];
  __shared__ double sJ[4][8], sG[4][24], sFp[4][8][9], sF[4][8][8][3];
  __shared__ HgoPoint sP[4][8];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * 4 + w;
  const bool live = e < A.n_elems;
  const double* m = live ? A.mat + 7 * A.elem_mat[e] : A.mat;
  const int kind = live ? (int)m[0] : -1;
  const bool hgo = kind == 1, lin = kind == 0;
  if (live && l < 24) {
    const int64_t nd = A.hex8[e * 8 + l / 3];
    sX[w][l] = A.xyz[nd * 3 + l % 3];
    sU[w][l] = A.U ? A.U[nd * 3 + l % 3] : 0.0;
  }
  __syncthreads();
  if (live && l < 8) {
    double Jm[9];
    for (int d = 0; d < 3; ++d)
      for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int a = 0; a < 8; ++a) s += sX[w][3 * a + d] * dshape(a, k, l);
        Jm[3 * d + k] = s;
      }
    double det;
    inv3(Jm, sInv[w][l], &det);
    sDet[w][l] = det;
  }
  __syncthreads();
  if (live) {
    const int gp = l >> 3, a = l & 7;
    for (int d = 0; d < 3; ++d) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += dshape(a, k, gp) * sInv[w][gp][3 * k + d];
      sdN[w][gp][a][d] = s;
    }
  }
  __syncthreads();
  // HGO stage 1: deformation gradient and J at every Gauss point
  if (hgo && l < 8) {
    const int gp = l;
    double F[9];
    for (int i = 0; i < 3; ++i)
      for (int J = 0; J < 3; ++J) {
        double s = (i == J) ? 1.0 : 0.0;
        for (int q = 0; q < 8; ++q) s += sU[w][3 * q + i] * sdN[w][gp][q][J];
        F[3 * i + J] = s;
      }
    double Fi[9], detF;
    inv3(F, Fi, &detF);
    // an element inverted by U (det F <= 0) has no strain energy: record it
    // (the host rejects the state) and keep the arithmetic finite
    if (!(detF > 0.0)) {
      if (A.inverted) atomicMin(A.inverted, (int)e);
      detF = 1.0;
      for (int k = 0; k < 9; ++k) F[k] = (k % 4 == 0) ? 1.0 : 0.0;
    }
    sJ[w][gp] = detF;
    for (int k = 0; k < 9; ++k) sFp[w][gp][k] = F[k];
  }
  __syncthreads();
  // HGO stage 2: element pressure, point stresses/tangents, g vector
  double V = 0.0, p = 0.0;
  if (hgo) {
    double v = 0.0;
    for (int gp = 0; gp < 8; ++gp) {
      V += sDet[w][gp];
      v += sDet[w][gp] * sJ[w][gp];
    }
    p = m[6] * (v / V - 1.0);
    if (l < 8) {
      const double* a1 = A.fibers + e * 6;
      hgo_point(sFp[w][l], sJ[w][l], p, a1, a1 + 3, m[3], m[4], m[5], sP[w][l]);
    }
    if (l < 24) {   // g_a = int J F^{-T} grad N_a, node l/3, component l%3
      const int q = l / 3, i = l % 3;
      double s = 0.0;
      for (int gp = 0; gp < 8; ++gp) {
        double Fi[9], dF;
        inv3(sFp[w][gp], Fi, &dF);
        double t = 0.0;
        for (int I = 0; I < 3; ++I) t += Fi[3 * I + i] * sdN[w][gp][q][I];
        s += sDet[w][gp] * sJ[w][gp] * t;
      }
      sG[w][l] = s;
    }
  }
  __syncthreads();
  const int a = l >> 3, b = l & 7;
  double K[9];
  for (int k = 0; k < 9; ++k) K[k] = 0.0;
  if (lin) {
    const double E = m[1], nu = m[2];
    const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E / (2.0 * (1.0 + nu));
    for (int gp = 0; gp < 8; ++gp) {
      const double* na = sdN[w][gp][a];
      const double* nb = sdN[w][gp][b];
      const double wt = sDet[w][gp];
      const double dot = na[0] * nb[0] + na[1] * nb[1] + na[2] * nb[2];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          K[3 * i + j] += wt * (lam * na[i] * nb[j] + mu * (na[j] * nb[i] + (i == j ? dot : 0.0)));
    }
  } else if (hgo) {
    for (int gp = 0; gp < 8; ++gp) {
      const HgoPoint& P = sP[w][gp];
      const double* na = sdN[w][gp][a];
      const double* nb = sdN[w][gp][b];
      const double wt = sDet[w][gp];
      double geo = 0.0;
      for (int I = 0; I < 3; ++I)
        for (int J = 0; J < 3; ++J) geo += na[I] * P.S[3 * I + J] * nb[J];
      double Ba[6][3], Bb[6][3];
      for (int al = 0; al < 6; ++al) {
        const int I = VA[al], J = VB[al];
        for (int i = 0; i < 3; ++i) {
          if (I == J) {
            Ba[al][i] = P.F[3 * i + I] * na[I];
            Bb[al][i] = P.F[3 * i + I] * nb[I];
          } else {
            Ba[al][i] = P.F[3 * i + I] * na[J] + P.F[3 * i + J] * na[I];
            Bb[al][i] = P.F[3 * i + I] * nb[J] + P.F[3 * i + J] * nb[I];
          }
        }
      }
      for (int j = 0; j < 3; ++j) {
        double cb[6];
        for (int al = 0; al < 6; ++al) {
          double s = 0.0;
          for (int be = 0; be < 6; ++be) s += P.CV[6 * al + be] * Bb[be][j];
          cb[al] = s;
        }
        for (int i = 0; i < 3; ++i) {
          double s = 0.0;
          for (int al = 0; al < 6; ++al) s += Ba[al][i] * cb[al];
          K[3 * i + j] += wt * (s + (i == j ? geo : 0.0));
        }
      }
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) K[3 * i + j] += m[6] / V * sG[w][3 * a + i] * sG[w][3 * b + j];
  }
  if (live) {
    double* out = A.Ke + e * 576 + (a * 8 + b) * 9;
    for (int k = 0; k < 9; ++k) out[k] = K[k];
  }
  // internal force: linear K_e u_e (reduced over b through LDS); HGO int F S grad N_a
  if (lin)
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
      for (int j = 0; j < 3; ++j) s += K[3 * i + j] * sU[w][3 * b + j];
      sF[w][a][b][i] = s;
    }
  __syncthreads();
  if (live && b == 0) {
    for (int i = 0; i < 3; ++i) {
      double fb = 0.0, fi = 0.0;
      if (A.body)
        for (int gp = 0; gp < 8; ++gp) fb += sDet[w][gp] * shape(a, gp) * A.body[e * 3 + i];
      if (lin) {
        for (int q = 0; q < 8; ++q) fi += sF[w][a][q][i];
      } else {
        for (int gp = 0; gp < 8; ++gp) {
          const HgoPoint& P = sP[w][gp];
          double t = 0.0;
          for (int J = 0; J < 3; ++J) {
            double FS = 0.0;
            for (int I = 0; I < 3; ++I) FS += P.F[3 * i + I] * P.S[3 * I + J];
            t += FS * sdN[w][gp][a][J];
          }
          fi += sDet[w][gp] * t;
        }
      }
      A.fbody[e * 24 + 3 * a + i] = fb;
      A.fint[e * 24 + 3 * a + i] = fi;
    }
  }
}

// ---------------------------------------------------------------------------
// Q2 elements (27-node triquadratic hexahedra, node a = i + 3j + 9k at
// reference point (i-1, j-1, k-1)), with the same materials as above and, for
// HGO, the same P0 condensation (the Q2-P0 pair of section 3.2): Jbar is the
// element's mean dilatation over its 3x3x3 Gauss points.  One 128-thread
// workgroup per element: threads share the Gauss-point data in LDS, and the
// 378 node-pair blocks a <= b are spread over the threads (the tangent is
// symmetric: the bilinear form of linear elasticity, and the second
// derivative of the HGO energy), each block stored with its transpose.

// Threads per Q2 element: the 378 node-pair blocks take three rounds of 128
// (98% of the threads busy; with 256, two rounds, the second half empty).
// Two waves per SIMD (at most 256 registers, 24 of them spilled) measured
// 3.63 ms for the 16,384 elements of the Q2 tube, against 5.12 ms at one wave
// per SIMD without spills and 4.15 ms with 256 threads.
constexpr int E27_T = 128;

// N_a and dN_a/dxi at Gauss point q = gi + 3 gj + 9 gk.
__device__ __forceinline__ void shape27(int a, int q, double* N, double dN[3]) {
  double L[3], dL[3];
  const int ia[3] = {a % 3, (a / 3) % 3, a / 9}, iq[3] = {q % 3, (q / 3) % 3, q / 9};
  for (int d = 0; d < 3; ++d) {
    const double x = gp3(iq[d]);
    L[d] = lag3(ia[d], x);
    dL[d] = dlag3(ia[d], x);
  }
  *N = L[0] * L[1] * L[2];
  dN[0] = dL[0] * L[1] * L[2];
  dN[1] = L[0] * dL[1] * L[2];
  dN[2] = L[0] * L[1] * dL[2];
}

__global__ __launch_bounds__(E27_T, 2) void k_elements27(AsmArgs A) {
  __shared__ double sX[81], sU[81], sInv[27][9], sW[27], sdN[27][27][3];
  __shared__ double sJ[27], sFp[27][9], sFi[27][9], sG[81], sSig[27][9];
  __shared__ HgoPoint sP[27];
  const int64_t e = blockIdx.x;
  const int t = threadIdx.x;
  const double* m = A.mat + 7 * A.elem_mat[e];
  const int kind = (int)m[0];
  const bool hgo = kind == 1, lin = kind == 0;
  if (t < 81) {
    const int64_t nd = A.hex8[e * 27 + t / 3];
    sX[t] = A.xyz[nd * 3 + t % 3];
    sU[t] = A.U ? A.U[nd * 3 + t % 3] : 0.0;
  }
  __syncthreads();
  // Jacobian dX/dxi, its inverse, and the quadrature weight w_q det J at each point
  if (t < 27) {
    double Jm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 27; ++a) {
      double N, dxi[3];
      shape27(a, t, &N, dxi);
      for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 3; ++k) Jm[3 * d + k] += sX[3 * a + d] * dxi[k];
    }
    double det;
    inv3(Jm, sInv[t], &det);
    sW[t] = gw3(t % 3) * gw3((t / 3) % 3) * gw3(t / 9) * det;
  }
  __syncthreads();
  for (int pr = t; pr < 729; pr += E27_T) {   // dN_a/dX at point q
    const int q = pr / 27, a = pr % 27;
    double N, dxi[3];
    shape27(a, q, &N, dxi);
    for (int d = 0; d < 3; ++d) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += dxi[k] * sInv[q][3 * k + d];
      sdN[q][a][d] = s;
    }
  }
  __syncthreads();
  if (t < 27) {
    double G[9];   // Grad U
    for (int i = 0; i < 3; ++i)
      for (int J = 0; J < 3; ++J) {
        double s = 0.0;
        for (int a = 0; a < 27; ++a) s += sU[3 * a + i] * sdN[t][a][J];
        G[3 * i + J] = s;
      }
    if (hgo) {
      double F[9], Fi[9], detF;
      for (int k = 0; k < 9; ++k) F[k] = G[k] + ((k % 4 == 0) ? 1.0 : 0.0);
      inv3(F, Fi, &detF);
      // an element inverted by U (det F <= 0) has no strain energy: record it
      // (the host rejects the state) and keep the arithmetic finite
      if (!(detF > 0.0)) {
        if (A.inverted) atomicMin(A.inverted, (int)e);
        detF = 1.0;
        for (int k = 0; k < 9; ++k) F[k] = Fi[k] = (k % 4 == 0) ? 1.0 : 0.0;
      }
      sJ[t] = detF;
      for (int k = 0; k < 9; ++k) {
        sFp[t][k] = F[k];
        sFi[t][k] = Fi[k];
      }
    } else if (lin) {   // Cauchy stress lam tr(eps) I + 2 mu eps of the displacement
      const double E = m[1], nu = m[2];
      const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E / (2.0 * (1.0 + nu));
      const double tr = G[0] + G[4] + G[8];
      for (int i = 0; i < 3; ++i)
        for (int J = 0; J < 3; ++J) sSig[t][3 * i + J] = mu * (G[3 * i + J] + G[3 * J + i]) + (i == J ? lam * tr : 0.0);
    }
  }
  __syncthreads();
  // element pressure, point stresses and tangents, and g_a = int J F^{-T} grad N_a
  double V = 0.0, p = 0.0;
  if (hgo) {
    double v = 0.0;
    for (int q = 0; q < 27; ++q) {
      V += sW[q];
      v += sW[q] * sJ[q];
    }
    p = m[6] * (v / V - 1.0);
    if (t < 27) {
      const double* a1 = A.fibers + e * 6;
      hgo_point(sFp[t], sJ[t], p, a1, a1 + 3, m[3], m[4], m[5], sP[t]);
    }
    if (t < 81) {
      const int a = t / 3, i = t % 3;
      double s = 0.0;
      for (int q = 0; q < 27; ++q) {
        double tq = 0.0;
        for (int I = 0; I < 3; ++I) tq += sFi[q][3 * I + i] * sdN[q][a][I];
        s += sW[q] * sJ[q] * tq;
      }
      sG[t] = s;
    }
  }
  __syncthreads();
  double* Ke = A.Ke + e * 6561;
  for (int pr = t; pr < 378; pr += E27_T) {
    int a = 0, r = pr;
    while (r >= 27 - a) {
      r -= 27 - a;
      ++a;
    }
    const int b = a + r;
    double K[9];
    for (int k = 0; k < 9; ++k) K[k] = 0.0;
    if (lin) {
      const double E = m[1], nu = m[2];
      const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = E / (2.0 * (1.0 + nu));
      for (int q = 0; q < 27; ++q) {
        const double* na = sdN[q][a];
        const double* nb = sdN[q][b];
        const double wt = sW[q];
        const double dot = na[0] * nb[0] + na[1] * nb[1] + na[2] * nb[2];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            K[3 * i + j] += wt * (lam * na[i] * nb[j] + mu * (na[j] * nb[i] + (i == j ? dot : 0.0)));
      }
    } else if (hgo) {
      for (int q = 0; q < 27; ++q) {
        const HgoPoint& P = sP[q];
        const double* na = sdN[q][a];
        const double* nb = sdN[q][b];
        const double wt = sW[q];
        double geo = 0.0;
        for (int I = 0; I < 3; ++I)
          for (int J = 0; J < 3; ++J) geo += na[I] * P.S[3 * I + J] * nb[J];
        double Ba[6][3], Bb[6][3];
        for (int al = 0; al < 6; ++al) {
          const int I = VA[al], J = VB[al];
          for (int i = 0; i < 3; ++i) {
            if (I == J) {
              Ba[al][i] = P.F[3 * i + I] * na[I];
              Bb[al][i] = P.F[3 * i + I] * nb[I];
            } else {
              Ba[al][i] = P.F[3 * i + I] * na[J] + P.F[3 * i + J] * na[I];
              Bb[al][i] = P.F[3 * i + I] * nb[J] + P.F[3 * i + J] * nb[I];
            }
          }
        }
        for (int j = 0; j < 3; ++j) {
          double cb[6];
          for (int al = 0; al < 6; ++al) {
            double s = 0.0;
            for (int be = 0; be < 6; ++be) s += P.CV[6 * al + be] * Bb[be][j];
            cb[al] = s;
          }
          for (int i = 0; i < 3; ++i) {
            double s = 0.0;
            for (int al = 0; al < 6; ++al) s += Ba[al][i] * cb[al];
            K[3 * i + j] += wt * (s + (i == j ? geo : 0.0));
          }
        }
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K[3 * i + j] += m[6] / V * sG[3 * a + i] * sG[3 * b + j];
    }
    double* out = Ke + (a * 27 + b) * 9;
    for (int k = 0; k < 9; ++k) out[k] = K[k];
    if (a != b) {
      double* tr = Ke + (b * 27 + a) * 9;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) tr[3 * j + i] = K[3 * i + j];
    }
  }
  // internal force int P grad N_a (P = F S for HGO, the Cauchy stress for
  // linear elasticity) and body force int N_a b
  if (t < 81) {
    const int a = t / 3, i = t % 3;
    double fb = 0.0, fi = 0.0;
    for (int q = 0; q < 27; ++q) {
      if (A.body) {
        double N, dxi[3];
        shape27(a, q, &N, dxi);
        fb += sW[q] * N * A.body[e * 3 + i];
      }
      double tq = 0.0;
      if (hgo) {
        const HgoPoint& P = sP[q];
        for (int J = 0; J < 3; ++J) {
          double FS = 0.0;
          for (int I = 0; I < 3; ++I) FS += P.F[3 * i + I] * P.S[3 * I + J];
          tq += FS * sdN[q][a][J];
        }
      } else if (lin) {
        for (int J = 0; J < 3; ++J) tq += sSig[q][3 * i + J] * sdN[q][a][J];
      }
      fi += sW[q] * tq;
    }
    A.fbody[e * 81 + t] = fb;
    A.fint[e * 81 + t] = fi;
  }
}

void asm_elements(const AsmArgs& a, int any_hgo, hipStream_t s) {
  (void)any_hgo;
  if (!a.n_elems) return;
  if (a.npe == 27) hipLaunchKernelGGL(k_elements27, dim3((unsigned)a.n_elems), dim3(E27_T), 0, s, a);
  else hipLaunchKernelGGL(k_elements, dim3((unsigned)((a.n_elems + 3) / 4)), dim3(256), 0, s, a);
}

// Node-pair gather: K_i[(a,i),(b,j)] = sum over shared elements (fixed order).
// One thread per entry (i, j) of a node pair's 3x3 block, so the nine
// threads of a pair read each element block's 72 contiguous bytes together.
template <typename T>
__global__ void k_gather_local(GatherArgs G, T* arena) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * G.n_slots) return;
  const int64_t sl = t / 9;
  const int k = (int)(t % 9), i = k / 3, j = k % 3;
  const int la = G.ps_a[sl], lb = G.ps_b[sl], nbr = G.ps_nbr[sl];
  const int row = G.loc_pos[3 * la + i];
  if (row < 0) return;
  double K = 0.0;
  for (int c = G.ps_c0[sl]; c < G.ps_c1[sl]; ++c) {
    const int e = G.pc_e[c], ab = G.pc_ab[c];
    K += G.Ke[(int64_t)e * (9 * G.npe * G.npe) + ((ab & 255) * G.npe + (ab >> 8)) * 9 + k];
  }
  const SubInfo s = G.subs[G.loc_sub[la]];
  G.ell_val[(int64_t)(nbr * 3 + j) * G.NF + s.full_off + row] = K;
  const int col = G.loc_pos[3 * lb + j];
  if (col >= 0 && row >= col) {
    const int ti = row / TS, tj = col / TS;
    arena[s.tile_off + tidx3(ti, tj) * TS2 + (col % TS) * TS + (row % TS)] = (T)K;
  }
}

template <typename T>
void asm_gather(const GatherArgs& g, T* arena, hipStream_t s) {
  if (g.n_slots) hipLaunchKernelGGL(k_gather_local<T>, dim3((unsigned)((9 * g.n_slots + 255) / 256)), dim3(256), 0, s, g, arena);
}
template void asm_gather<double>(const GatherArgs&, double*, hipStream_t);
template void asm_gather<float>(const GatherArgs&, float*, hipStream_t);

// Local right-hand side: body_scale * f_body - int_scale * f_int + nodal share,
// minus the coupling to eliminated Dirichlet DOFs (classical variant).
__global__ void k_rhs(RhsArgs R) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * R.n_loc_nodes) return;
  const int64_t la = t / 3;
  const int i = (int)(t % 3);
  const int pos = R.loc_pos[t];
  if (pos < 0) return;
  const SubInfo s = R.subs[R.loc_sub[la]];
  const int sl = R.diag_slot[la];
  double fb = 0.0, fi = 0.0;
  for (int c = R.ps_c0[sl]; c < R.ps_c1[sl]; ++c) {
    const int e = R.pc_e[c], lq = R.pc_ab[c] & 255;
    fb += R.fbody[(int64_t)e * (3 * R.npe) + 3 * lq + i];
    if (R.int_scale != 0.0) fi += R.fint[(int64_t)e * (3 * R.npe) + 3 * lq + i];
  }
  double f = R.body_scale * fb - R.int_scale * fi;
  const int64_t g = R.loc_node[la];
  if (R.fnodal) f += R.nodal_scale * R.fnodal[3 * g + i] / R.loc_ncopy[la];
  const int64_t row = s.full_off + pos;
  for (int k = 0; k < R.ellw; ++k) {
    const int cc = R.ell_col[k * R.NF + row];
    if (cc == -1) break;   // the filled slots of a row form a prefix
    if (cc <= -2) f -= R.ell_val[k * R.NF + row] * R.dvals[-(cc + 2)];
  }
  R.f[row] = f;
}

void asm_rhs(const RhsArgs& r, hipStream_t s) {
  if (r.n_loc_nodes) hipLaunchKernelGGL(k_rhs, dim3((unsigned)((3 * r.n_loc_nodes + 255) / 256)), dim3(256), 0, s, r);
}

// Quadrilateral pressure faces.  NFN = 4: bilinear, corners (-1,-1), (1,-1),
// (1,1), (-1,1), 2x2 Gauss points of weight 1.  NFN = 9: biquadratic, node
// c = i + 3j at (i-1, j-1), 3x3 Gauss points.
template <int NFN>
struct FaceRule;
template <>
struct FaceRule<4> {
  static constexpr int NG = 2;
  __device__ static double pt(int g) { return g ? 0.57735026918962576451 : -0.57735026918962576451; }
  __device__ static double wt(int) { return 1.0; }
  __device__ static void shape(int c, double s, double t, double& N, double& ds, double& dt) {
    const double e1 = (c == 1 || c == 2) ? 1.0 : -1.0, e2 = c >= 2 ? 1.0 : -1.0;
    N = 0.25 * (1 + e1 * s) * (1 + e2 * t);
    ds = 0.25 * e1 * (1 + e2 * t);
    dt = 0.25 * e2 * (1 + e1 * s);
  }
};
template <>
struct FaceRule<9> {
  static constexpr int NG = 3;
  __device__ static double pt(int g) { return gp3(g); }
  __device__ static double wt(int g) { return gw3(g); }
  __device__ static void shape(int c, double s, double t, double& N, double& ds, double& dt) {
    const int i = c % 3, j = c / 3;
    N = lag3(i, s) * lag3(j, t);
    ds = dlag3(i, s) * lag3(j, t);
    dt = lag3(i, s) * dlag3(j, t);
  }
};

// Follower pressure on the current surface: f_a = -p int N_a (x,s x x,t) ds dt.
// One thread per node sums over its faces in a fixed order (no atomics).
template <int NFN>
__global__ __launch_bounds__(256) void k_pressure(PressureArgs P) {
  using R = FaceRule<NFN>;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P.n_nodes) return;
  double f[3] = {0, 0, 0};
  for (int k = P.pf_ptr[n]; k < P.pf_ptr[n + 1]; ++k) {
    const int64_t fc = P.pf_ent[k];
    const int64_t face = fc / NFN;
    const int cn = (int)(fc % NFN);
    double x[NFN][3];
#pragma unroll
    for (int q = 0; q < NFN; ++q) {
      const int64_t nd = P.pface[face * NFN + q];
      for (int d = 0; d < 3; ++d) x[q][d] = P.xyz[nd * 3 + d] + (P.U ? P.U[nd * 3 + d] : 0.0);
    }
    for (int g1 = 0; g1 < R::NG; ++g1)
      for (int g2 = 0; g2 < R::NG; ++g2) {
        const double h1 = R::pt(g1), h2 = R::pt(g2);
        double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0}, N, d1, d2;
    #pragma unroll
    for (int q = 0; q < NFN; ++q) {
          R::shape(q, h1, h2, N, d1, d2);
          for (int d = 0; d < 3; ++d) {
            t1[d] += x[q][d] * d1;
            t2[d] += x[q][d] * d2;
          }
        }
        const double nv[3] = {t1[1] * t2[2] - t1[2] * t2[1], t1[2] * t2[0] - t1[0] * t2[2],
                              t1[0] * t2[1] - t1[1] * t2[0]};
        R::shape(cn, h1, h2, N, d1, d2);
        const double pw = -P.pressure * (R::wt(g1) * R::wt(g2));
        for (int d = 0; d < 3; ++d) f[d] += pw * N * nv[d];
      }
  }
  for (int d = 0; d < 3; ++d) P.fnodal[3 * n + d] = f[d];
}

void asm_pressure(const PressureArgs& p, hipStream_t s) {
  if (!p.n_nodes) return;
  const dim3 grid((unsigned)((p.n_nodes + 255) / 256));
  if (p.nfn == 9) hipLaunchKernelGGL(k_pressure<9>, grid, dim3(256), 0, s, p);
  else hipLaunchKernelGGL(k_pressure<4>, grid, dim3(256), 0, s, p);
}

// Load stiffness of the follower pressure applied to a direction z: the
// derivative of f_a = -p int N_a (x,s x x,t) ds dt along x -> x + z is
//   out_a = -p int N_a (z,s x x,t + x,s x z,t) ds dt,
// with z,s and z,t interpolated from the nodal values of z like x,s and x,t.
// One thread per node sums over its faces in a fixed order (no atomics);
// Dirichlet DOFs (dmask) get 0.
template <int NFN>
__global__ __launch_bounds__(256) void k_pressure_dir(PressureArgs P, const double* __restrict__ z, const uint8_t* __restrict__ dmask,
                               double* __restrict__ out) {
  using R = FaceRule<NFN>;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P.n_nodes) return;
  double f[3] = {0, 0, 0};
  for (int k = P.pf_ptr[n]; k < P.pf_ptr[n + 1]; ++k) {
    const int64_t fc = P.pf_ent[k];
    const int64_t face = fc / NFN;
    const int cn = (int)(fc % NFN);
    double x[NFN][3], dz[NFN][3];
#pragma unroll
    for (int q = 0; q < NFN; ++q) {
      const int64_t nd = P.pface[face * NFN + q];
      for (int d = 0; d < 3; ++d) {
        x[q][d] = P.xyz[nd * 3 + d] + (P.U ? P.U[nd * 3 + d] : 0.0);
        dz[q][d] = z[nd * 3 + d];
      }
    }
    for (int g1 = 0; g1 < R::NG; ++g1)
      for (int g2 = 0; g2 < R::NG; ++g2) {
        const double h1 = R::pt(g1), h2 = R::pt(g2);
        double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0}, s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0}, N, d1, d2;
    #pragma unroll
    for (int q = 0; q < NFN; ++q) {
          R::shape(q, h1, h2, N, d1, d2);
          for (int d = 0; d < 3; ++d) {
            t1[d] += x[q][d] * d1;
            t2[d] += x[q][d] * d2;
            s1[d] += dz[q][d] * d1;
            s2[d] += dz[q][d] * d2;
          }
        }
        // s1 x t2 + t1 x s2
        const double nv[3] = {s1[1] * t2[2] - s1[2] * t2[1] + t1[1] * s2[2] - t1[2] * s2[1],
                              s1[2] * t2[0] - s1[0] * t2[2] + t1[2] * s2[0] - t1[0] * s2[2],
                              s1[0] * t2[1] - s1[1] * t2[0] + t1[0] * s2[1] - t1[1] * s2[0]};
        R::shape(cn, h1, h2, N, d1, d2);
        const double pw = -P.pressure * (R::wt(g1) * R::wt(g2));
        for (int d = 0; d < 3; ++d) f[d] += pw * N * nv[d];
      }
  }
  for (int d = 0; d < 3; ++d) out[3 * n + d] = dmask[3 * n + d] ? 0.0 : f[d];
}

void asm_pressure_dir(const PressureArgs& p, const double* z, const uint8_t* dmask, double* out, hipStream_t s) {
  if (!p.n_nodes) return;
  const dim3 grid((unsigned)((p.n_nodes + 255) / 256));
  if (p.nfn == 9) hipLaunchKernelGGL(k_pressure_dir<9>, grid, dim3(256), 0, s, p, z, dmask, out);
  else hipLaunchKernelGGL(k_pressure_dir<4>, grid, dim3(256), 0, s, p, z, dmask, out);
}

// ---------------------------------------------------------------------------
// Rigid-body kernel of each floating subdomain: translations and rotations
// about the current centroid (rotations kept only if K annihilates them, for
// stressed tangents); Gram-Schmidt (two passes, FP64) on the interface rows
// gives an orthonormal Rb = R_b T; the full basis R T is used for G, e and
// the recovery of the displacements.
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

static_assert(ELLW_Q1 % 9 == 0 && ELLW_Q2 % 9 == 0, "the rotation test reads slots in groups of 9");
__global__ __launch_bounds__(256) void k_modes_setup(ModesArgs M) {
  __shared__ double red[256];
  __shared__ double cen[3];
  const int sid = blockIdx.x;
  const SubInfo s = M.subs[sid];
  const int64_t n = (int64_t)s.nt * TS;
  double* rf = M.rfull + s.full_off * 6;
  double* W = M.work + s.full_off * 6;
  const int tid = threadIdx.x;
  if (!s.floating) {
    for (int64_t p = tid; p < n * 6; p += 256) rf[p] = 0.0;
    for (int64_t p = tid; p < (int64_t)s.nt_b * TS * 6; p += 256) M.rb[s.b_off * 6 + p] = 0.0;
    if (tid == 0) M.n_modes[sid] = 0;
    return;
  }
  for (int d = 0; d < 3; ++d) {
    double acc = 0.0;
    for (int q = tid; q < s.n_nodes; q += 256) {
      const int64_t g = M.loc_node[s.node_off + q];
      acc += M.xyz[g * 3 + d] + (M.U ? M.U[g * 3 + d] : 0.0);
    }
    const double tot = block_sum(acc, red);
    if (tid == 0) cen[d] = tot / s.n_nodes;
  }
  __syncthreads();
  for (int64_t p = tid; p < n; p += 256) {
    const int ln = M.fpos_lnode[s.full_off + p];
    double r[6] = {0, 0, 0, 0, 0, 0};
    if (ln >= 0) {
      const int comp = M.fpos_comp[s.full_off + p];
      const int64_t g = M.loc_node[ln];
      double x[3];
      for (int d = 0; d < 3; ++d) x[d] = M.xyz[g * 3 + d] + (M.U ? M.U[g * 3 + d] : 0.0) - cen[d];
      r[comp] = 1.0;
      // rotation about x: (0,-z,y); about y: (z,0,-x); about z: (-y,x,0)
      if (comp == 0) { r[4] = x[2]; r[5] = -x[1]; }
      if (comp == 1) { r[3] = -x[2]; r[5] = x[0]; }
      if (comp == 2) { r[3] = x[1]; r[4] = -x[0]; }
    }
    for (int k = 0; k < 6; ++k) W[p * 6 + k] = r[k];
  }
  __syncthreads();
  // A classical subdomain touching the Dirichlet boundary (floating == 2): its
  // kernel is the set of rigid modes that vanish on its Dirichlet DOFs, the
  // null space of R_D (the six modes at those DOFs).  With the rotations
  // scaled by the subdomain's radius Lr, the 6x6 Gram matrix R_D^T R_D is
  // diagonalised (cyclic Jacobi, one thread) and W is rotated onto its
  // eigenvectors, smallest eigenvalue first: the columns with eigenvalue at
  // most 1e-10 of the largest span the kernel.
  __shared__ int n_cand;
  if (s.floating == 2) {
    __shared__ double Mg[6][6], Ev[6][6];
    double lr = 0.0;
    for (int q = tid; q < s.n_nodes; q += 256) {
      const int64_t g = M.loc_node[s.node_off + q];
      for (int d = 0; d < 3; ++d) {
        const double x = M.xyz[g * 3 + d] + (M.U ? M.U[g * 3 + d] : 0.0) - cen[d];
        lr += x * x;
      }
    }
    const double Lr = sqrt(block_sum(lr, red) / s.n_nodes);
    const double il = Lr > 0.0 ? 1.0 / Lr : 1.0;
    for (int a = 0; a < 6; ++a)
      for (int b = a; b < 6; ++b) {
        double acc = 0.0;
        for (int q = tid; q < s.n_nodes; q += 256) {
          const int64_t g = M.loc_node[s.node_off + q];
          double x[3];
          for (int d = 0; d < 3; ++d) x[d] = (M.xyz[g * 3 + d] + (M.U ? M.U[g * 3 + d] : 0.0) - cen[d]) * il;
          for (int c = 0; c < 3; ++c) {
            if (!M.dmask[g * 3 + c]) continue;
            double r[6] = {0, 0, 0, 0, 0, 0};
            r[c] = 1.0;
            if (c == 0) { r[4] = x[2]; r[5] = -x[1]; }
            if (c == 1) { r[3] = -x[2]; r[5] = x[0]; }
            if (c == 2) { r[3] = x[1]; r[4] = -x[0]; }
            acc += r[a] * r[b];
          }
        }
        const double v = block_sum(acc, red);
        if (tid == 0) Mg[a][b] = Mg[b][a] = v;
      }
    if (tid == 0) {
      double A[6][6], V[6][6];
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
          A[a][b] = Mg[a][b];
          V[a][b] = a == b ? 1.0 : 0.0;
        }
      for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int a = 0; a < 6; ++a)
          for (int b = 0; b < 6; ++b) (a == b ? dia : off) += A[a][b] * A[a][b];
        if (off <= 1e-32 * dia) break;
        for (int a = 0; a < 5; ++a)
          for (int b = a + 1; b < 6; ++b) {
            if (A[a][b] == 0.0) continue;
            const double th = 0.5 * (A[b][b] - A[a][a]) / A[a][b];
            const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
            for (int k = 0; k < 6; ++k) {
              const double aka = A[k][a], akb = A[k][b];
              A[k][a] = c * aka - sn * akb;
              A[k][b] = sn * aka + c * akb;
            }
            for (int k = 0; k < 6; ++k) {
              const double aak = A[a][k], abk = A[b][k];
              A[a][k] = c * aak - sn * abk;
              A[b][k] = sn * aak + c * abk;
            }
            for (int k = 0; k < 6; ++k) {
              const double vka = V[k][a], vkb = V[k][b];
              V[k][a] = c * vka - sn * vkb;
              V[k][b] = sn * vka + c * vkb;
            }
          }
      }
      // eigenvalues ascending; coefficients of the unscaled modes (rotation rows / Lr)
      int ord[6] = {0, 1, 2, 3, 4, 5};
      for (int a = 1; a < 6; ++a)
        for (int b = a; b > 0 && A[ord[b]][ord[b]] < A[ord[b - 1]][ord[b - 1]]; --b) {
          const int t = ord[b];
          ord[b] = ord[b - 1];
          ord[b - 1] = t;
        }
      const double lmax = A[ord[5]][ord[5]];
      int nk = 0;
      for (int a = 0; a < 6; ++a) nk += A[ord[a]][ord[a]] <= 1e-10 * lmax;
      n_cand = nk;
      for (int j = 0; j < 6; ++j)
        for (int k = 0; k < 6; ++k) Ev[j][k] = V[j][ord[k]] * (j >= 3 ? il : 1.0);
    }
    __syncthreads();
    for (int64_t p = tid; p < n; p += 256) {
      double r[6];
      for (int k = 0; k < 6; ++k) {
        double acc = 0.0;
        for (int j = 0; j < 6; ++j) acc += W[p * 6 + j] * Ev[j][k];
        r[k] = acc;
      }
      for (int k = 0; k < 6; ++k) W[p * 6 + k] = r[k];
    }
  } else if (tid == 0) {
    n_cand = 6;
  }
  __syncthreads();
  if (tid == 0) M.n_modes[sid] = n_cand;   // the candidate count, until k_modes_finish
}

// The rotation test's sweep over the ELL rows, split over MODES_CH
// workgroups per subdomain: each sums, over its rows, ||K row||^2 and, for
// every candidate k, |(K r_k)_p|^2 and r_k,p^2 (slots in slot order, groups
// of 9 loaded together); k_modes_finish adds the chunks in order.
__global__ __launch_bounds__(256) void k_modes_sweep(ModesArgs M) {
  __shared__ double red[256];
  const int sid = blockIdx.x;
  const SubInfo s = M.subs[sid];
  if (!s.floating) return;
  const int64_t n = (int64_t)s.nt * TS;
  const double* W = M.work + s.full_off * 6;
  const int tid = threadIdx.x;
  const bool partial = s.floating == 2;
  const int k_first = partial ? 0 : 3, k_last = partial ? M.n_modes[sid] : 6;
  const int64_t chunk = (n + MODES_CH - 1) / MODES_CH;
  const int64_t lo = (int64_t)blockIdx.y * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double kf = 0.0, kr[6] = {0, 0, 0, 0, 0, 0}, rr[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t p = lo + tid; p < hi; p += 256) {
    const int64_t row = s.full_off + p;
    double y[6] = {0, 0, 0, 0, 0, 0};
    for (int q0 = 0; q0 < M.ellw; q0 += 9) {
      int c[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) c[i] = M.ell_col[(int64_t)(q0 + i) * M.NF + row];
      if (c[0] == -1) break;   // the filled slots of a row form a prefix
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        if (c[i] < 0) continue;
        const double v = M.ell_val[(int64_t)(q0 + i) * M.NF + row];
        kf += v * v;
        const double* w = W + (int64_t)c[i] * 6;
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (k >= k_first && k < k_last) y[k] += v * w[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (k >= k_first && k < k_last) {
        kr[k] += y[k] * y[k];
        rr[k] += W[p * 6 + k] * W[p * 6 + k];
      }
  }
  double* out = M.part + ((int64_t)sid * MODES_CH + blockIdx.y) * 13;
  const double t = block_sum(kf, red);
  if (tid == 0) out[0] = t;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double a = block_sum(kr[k], red), b = block_sum(rr[k], red);
    if (tid == 0) {
      out[1 + k] = a;
      out[7 + k] = b;
    }
  }
}

__global__ __launch_bounds__(256) void k_modes_finish(ModesArgs M) {
  __shared__ double red[256];
  __shared__ double T[6][6];
  __shared__ int sel[6], nsel;
  const int sid = blockIdx.x;
  const SubInfo s = M.subs[sid];
  if (!s.floating) return;
  const int64_t n = (int64_t)s.nt * TS;
  double* rf = M.rfull + s.full_off * 6;
  const double* W = M.work + s.full_off * 6;
  const int tid = threadIdx.x;
  const int n_cand = M.n_modes[sid];
  __shared__ int failed[6], nfail;
  // candidates: floating == 1 keeps the translations (in the kernel of every
  // tangent) and tests the rotations; floating == 2 tests its n_cand columns
  const bool partial = s.floating == 2;
  const int k_first = partial ? 0 : 3, k_last = partial ? n_cand : 6;
  if (tid == 0) {
    nsel = k_first;
    nfail = 0;
    for (int k = 0; k < k_first; ++k) sel[k] = k;
  }
  __syncthreads();
  if (M.test_rotations) {
    if (tid == 0) {   // the sweep's chunks, added in chunk order
      const double* pt = M.part + (int64_t)sid * MODES_CH * 13;
      double v[13];
      for (int q = 0; q < 13; ++q) v[q] = 0.0;
      for (int c = 0; c < MODES_CH; ++c)
        for (int q = 0; q < 13; ++q) v[q] += pt[c * 13 + q];
      const double knorm = sqrt(v[0]);
      for (int k = k_first; k < k_last; ++k) {
        if (sqrt(v[1 + k]) <= M.kernel_tol * knorm * sqrt(v[7 + k])) sel[nsel++] = k;
        else failed[nfail++] = k;
      }
    }
    __syncthreads();
    // kernel modes first, then the candidates the stressed tangent does not
    // annihilate, then (floating == 2) the modes outside the kernel
    if (tid == 0) {
      for (int q = 0; q < nfail; ++q) sel[nsel + q] = failed[q];
      for (int k = k_last; k < 6; ++k) sel[nsel + nfail + (k - k_last)] = k;
    }
    __syncthreads();
  } else {
    if (tid == 0) {
      nsel = k_last;
      for (int k = 0; k < 6; ++k) sel[k] = k;
    }
    __syncthreads();
  }
  const int n_kernel = nsel;
  const int m = 6;   // all six rigid modes regularise; the first n_kernel span the kernel
  // two-pass classical Gram-Schmidt on the interface rows; Q kept in rb
  const int64_t b0 = (int64_t)s.nt_i * TS, nb = (int64_t)s.nt_b * TS;
  double* Q = M.rb + s.b_off * 6;
  for (int64_t p = tid; p < nb * 6; p += 256) Q[p] = 0.0;
  if (tid < 36) T[tid / 6][tid % 6] = (tid / 6 == tid % 6) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    for (int64_t p = tid; p < nb; p += 256) Q[p * 6 + k] = W[(b0 + p) * 6 + sel[k]];
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int j = 0; j < k; ++j) {
        double acc = 0.0;
        for (int64_t p = tid; p < nb; p += 256) acc += Q[p * 6 + j] * Q[p * 6 + k];
        const double cj = block_sum(acc, red);
        for (int64_t p = tid; p < nb; p += 256) Q[p * 6 + k] -= cj * Q[p * 6 + j];
        if (tid < 6) T[tid][k] -= cj * T[tid][j];
        __syncthreads();
      }
    }
    double acc = 0.0;
    for (int64_t p = tid; p < nb; p += 256) acc += Q[p * 6 + k] * Q[p * 6 + k];
    const double nrm = sqrt(block_sum(acc, red));
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int64_t p = tid; p < nb; p += 256) Q[p * 6 + k] *= inv;
    if (tid < 6) T[tid][k] *= inv;
    __syncthreads();
  }
  // full basis R T; a partially constrained subdomain regularises with its
  // kernel modes only, so its other columns are zero
  const int m_keep = partial ? n_kernel : m;
  for (int64_t p = tid; p < nb * 6; p += 256)
    if ((int)(p % 6) >= m_keep) Q[p] = 0.0;
  for (int64_t p = tid; p < n; p += 256) {
    for (int k = 0; k < 6; ++k) {
      double acc = 0.0;
      if (k < m_keep)
        for (int j = 0; j < m; ++j) acc += W[p * 6 + sel[j]] * T[j][k];
      rf[p * 6 + k] = acc;
    }
  }
  if (tid == 0) M.n_modes[sid] = n_kernel;
}

void asm_modes(const ModesArgs& m, hipStream_t s) {
  hipLaunchKernelGGL(k_modes_setup, dim3(m.n_sub), dim3(256), 0, s, m);
  if (m.test_rotations) hipLaunchKernelGGL(k_modes_sweep, dim3(m.n_sub, MODES_CH), dim3(256), 0, s, m);
  hipLaunchKernelGGL(k_modes_finish, dim3(m.n_sub), dim3(256), 0, s, m);
}

// Coarse matrix Q = G^T G with G = [B_i Rb_i]: block (s, t), s >= t, sums
// c_s c_t Rb_s[b_s] Rb_t[b_t]^T over the multiplier rows the two share
// (interleaved over seven thread groups, then summed in group order); written
// into the lower tiles of the dense coarse matrix.
__global__ __launch_bounds__(256) void k_coarse_q(CoarseArgs C) {
  // 36 entries (a, b) of the 6x6 block of one subdomain pair, each summed by
  // QGROUPS threads over interleaved shared rows, then in a fixed order
  constexpr int QGROUPS = 7;
  __shared__ double part[QGROUPS][36];
  const int k = blockIdx.x;
  const int s = C.qp_s[k], t = C.qp_t[k];
  const SubInfo Ss = C.subs[s], St = C.subs[t];
  const int ab = threadIdx.x % 36, g = threadIdx.x / 36;
  const int a = ab / 6, b = ab % 6;
  double acc = 0.0;
  if (g < QGROUPS && a < Ss.n_modes && b < St.n_modes) {
    const int q0 = C.qp_ptr[k], q1 = C.qp_ptr[k + 1];
    for (int q = q0 + g; q < q1; q += QGROUPS)
      acc += C.qe_c[q] * C.rb[C.qe_bs[q] * 6 + a] * C.rb[C.qe_bt[q] * 6 + b];
  }
  if (g < QGROUPS) part[g][ab] = acc;
  __syncthreads();
  if (threadIdx.x >= 36 || a >= Ss.n_modes || b >= St.n_modes) return;
  double v = 0.0;
  for (int h = 0; h < QGROUPS; ++h) v += part[h][ab];
  const int row = Ss.coarse_off + a, col = St.coarse_off + b;
  if (row < col) return;
  C.q[tidx3(row / TS, col / TS) * TS2 + (col % TS) * TS + (row % TS)] = v;
}

void asm_coarse(const CoarseArgs& c, hipStream_t s) {
  if (c.n_pairs) hipLaunchKernelGGL(k_coarse_q, dim3(c.n_pairs), dim3(256), 0, s, c);
}

}  // namespace feti

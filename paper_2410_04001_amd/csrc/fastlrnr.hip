// FastLRNR construction on the device (arXiv 2410.04001, Section 2.2, eq. 2.7,
// and the construction of Section 4): FP64 snapshots of the hidden states, POD
// basis Xi (leading left singular vectors of the snapshot matrix, by one-sided
// Jacobi (Hestenes) SVD, which keeps small singular vectors accurate), DEIM
// indices P (Chaturantabut & Sorensen greedy; ties to the smallest index) and
// the reduced operators
//   U_hat = P^T U,  b_hat = P^T b,  V_hat^{l+1} = (V^{(l+1)T} Xi (P^T Xi)^{-1})^T.
// The reduced network is an LRNR whose hidden widths are r_hat, so the fused
// kernel runs it unchanged.  This is set-up work; it allocates its own scratch.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "lrnr_bias.h"

struct fastlrnr_handle {
  lrnr_net net;           // reduced net; U, V, b point at the buffers below
  float* U = nullptr;
  float* V = nullptr;
  float* b = nullptr;
  int32_t* Pd = nullptr;  // device copy of P
  std::vector<int32_t> P; // concatenated indices of hidden layers 1..L-1
};

namespace lrnr {

constexpr int kSelThreads = 1024;

// Value-only forward of the LRNR at the snapshot points in FP64; writes the
// hidden states z^l (l = 1..L-1) neuron-major: Zt_l[w][col], col = i_s * n_snap + j.
__global__ void snapshot_kernel(KNet net, const float* __restrict__ s_snap, int n_s,
                                const float* __restrict__ xt, int64_t n_snap,
                                double* __restrict__ Zt, int64_t ncols) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncols) return;
  const int is = (int)(col / n_snap);
  const int64_t j = col - (int64_t)is * n_snap;
  const float* s = s_snap + (int64_t)is * net.r_total;
  const double x = xt[2 * j], t = xt[2 * j + 1];
  double y[LRNR_MAX_RANK], yn[LRNR_MAX_RANK];
  const int r1 = net.r[1];
  const float* V1 = net.V + net.offV[1];
#pragma unroll
  for (int k = 0; k < LRNR_MAX_RANK; ++k)
    y[k] = k < r1 ? (double)V1[k] * x + (double)V1[r1 + k] * t : 0.0;
  int64_t zoff = 0;
  for (int l = 1; l <= net.L - 1; ++l) {
    const int W = net.M[l], rl = net.r[l], ro = net.r[l + 1];
    const float* U = net.U + net.offU[l];
    const float* V = net.V + net.offV[l + 1];
    const float* b = net.b + net.offB[l];
    const float* sl = s + net.offS[l];
#pragma unroll
    for (int k = 0; k < LRNR_MAX_RANK; ++k) {
      yn[k] = 0.0;
      if (k < rl) y[k] *= (double)sl[k];
    }
    double* Zl = Zt + zoff + col;
    for (int w = 0; w < W; ++w) {
      double a = b[w];
#pragma unroll
      for (int k = 0; k < LRNR_MAX_RANK; ++k)
        if (k < rl) a += (double)U[w * rl + k] * y[k];
      const double z = sin(a);
      Zl[(int64_t)w * ncols] = z;
#pragma unroll
      for (int k = 0; k < LRNR_MAX_RANK; ++k)
        if (k < ro) yn[k] += (double)V[w * ro + k] * z;
    }
#pragma unroll
    for (int k = 0; k < LRNR_MAX_RANK; ++k) y[k] = yn[k];
    zoff += ncols * W;
  }
}

struct SelShared {
  double val[kSelThreads];
  int idx[kSelThreads];
};

// Index in [0, n) maximising |v[i*stride]|; ties go to the smallest index.
__device__ int wg_argmax_abs(const double* __restrict__ v, int n, int64_t stride,
                             SelShared& sh) {
  const int tid = threadIdx.x;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int i = tid; i < n; i += blockDim.x) {
    const double a = fabs(v[i * stride]);
    if (a > best) {
      best = a;
      bi = i;
    }
  }
  sh.val[tid] = best;
  sh.idx[tid] = bi;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) {
      const double ov = sh.val[tid + off];
      const int oi = sh.idx[tid + off];
      if (ov > sh.val[tid] || (ov == sh.val[tid] && oi < sh.idx[tid])) {
        sh.val[tid] = ov;
        sh.idx[tid] = oi;
      }
    }
    __syncthreads();
  }
  const int r = sh.idx[0];
  __syncthreads();
  return r;
}

// Solves A X = B in place (A: n x n, row stride lda; B: n x nrhs, row stride
// ldb) by Gaussian elimination with partial pivoting.  Returns false when a
// pivot is zero.
__device__ bool wg_solve(double* __restrict__ A, int n, int lda, double* __restrict__ B,
                         int nrhs, int ldb, SelShared& sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < n; ++k) {
    const int piv = k + wg_argmax_abs(A + (int64_t)k * lda + k, n - k, lda, sh);
    if (A[(int64_t)piv * lda + k] == 0.0) return false;
    if (piv != k) {
      for (int j = tid; j < n + nrhs; j += nt) {
        if (j < n) {
          const double t = A[(int64_t)k * lda + j];
          A[(int64_t)k * lda + j] = A[(int64_t)piv * lda + j];
          A[(int64_t)piv * lda + j] = t;
        } else {
          const int c = j - n;
          const double t = B[(int64_t)k * ldb + c];
          B[(int64_t)k * ldb + c] = B[(int64_t)piv * ldb + c];
          B[(int64_t)piv * ldb + c] = t;
        }
      }
      __syncthreads();
    }
    const double inv = 1.0 / A[(int64_t)k * lda + k];
    for (int i = k + 1 + tid; i < n; i += nt) A[(int64_t)i * lda + k] *= inv;
    __syncthreads();
    const int rows = n - k - 1, cols = n - k - 1 + nrhs;
    for (int e = tid; e < rows * cols; e += nt) {
      const int i = k + 1 + e / cols, c = e % cols;
      const double m = A[(int64_t)i * lda + k];
      if (c < n - k - 1) {
        const int j = k + 1 + c;
        A[(int64_t)i * lda + j] -= m * A[(int64_t)k * lda + j];
      } else {
        const int cc = c - (n - k - 1);
        B[(int64_t)i * ldb + cc] -= m * B[(int64_t)k * ldb + cc];
      }
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const double inv = 1.0 / A[(int64_t)k * lda + k];
    for (int c = tid; c < nrhs; c += nt) B[(int64_t)k * ldb + c] *= inv;
    __syncthreads();
    for (int e = tid; e < k * nrhs; e += nt) {
      const int i = e / nrhs, c = e % nrhs;
      B[(int64_t)i * ldb + c] -= A[(int64_t)i * lda + k] * B[(int64_t)k * ldb + c];
    }
    __syncthreads();
  }
  return true;
}

struct SelArgs {
  int M, r_hat, ro;           // layer width, reduced width, next rank r_{l+1}
  int rl;                     // this layer's rank r_l
  double* Zt;                 // [M][ncols] snapshot rows = columns of A = Z^T; destroyed
  int64_t ncols;
  double* E;                  // [M][M] right singular vectors of A (columns)
  double* Xi;                 // [M][r_hat]
  double* A;                  // [r_hat][r_hat] (+ one row) scratch
  double* R;                  // [max(M, r_hat * ro)] scratch
  int* rank;                  // [M]
  int* P;                     // [r_hat] out (device)
  const float* U;             // U^l [M][rl]
  const float* b;             // b^l [M]
  const float* Vn;            // V^{l+1} [M][ro]
  float* Uh;                  // [r_hat][rl] out
  float* bh;                  // [r_hat] out
  float* Vh;                  // [r_hat][ro] out
  int* status;                // set to 1 on breakdown
  int qdeim;                  // index selection: 0 DEIM, 1 Q-DEIM
};

__global__ __launch_bounds__(kSelThreads) void select_kernel(SelArgs a) {
  __shared__ SelShared sh;
  __shared__ double cs_c[LRNR_MAX_WIDTH / 2 + 1], cs_s[LRNR_MAX_WIDTH / 2 + 1];
  __shared__ int pr_p[LRNR_MAX_WIDTH / 2 + 1], pr_q[LRNR_MAX_WIDTH / 2 + 1];
  __shared__ double gsum[kSelThreads][3];
  __shared__ int any_rot;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int M = a.M, rh = a.r_hat;
  const int64_t nc = a.ncols;

  // ---- one-sided Jacobi SVD of A = Z^T (its columns are the rows of Zt) ---
  // Rotations of column pairs, in round-robin order, until every pair is
  // orthogonal to 1e-15 relative; E accumulates them (A E = Q Sigma), so the
  // columns of E are the left singular vectors of Z.
  for (int e = tid; e < M * M; e += nt) a.E[e] = (e / M == e % M) ? 1.0 : 0.0;
  __syncthreads();
  const int n = (M + 1) & ~1;  // even count; index M (when M is odd) is a bye
  const int npair = n / 2;
  int G = 1;                   // threads per pair (power of two)
  while (G * 2 * npair <= nt) G *= 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int round = 0; round < n - 1; ++round) {
      const int k = tid / G, gl = tid % G;
      int p = 0, q = 0;
      if (k < npair) {
        p = k == 0 ? 0 : ((k - 1 + round) % (n - 1)) + 1;
        const int kq = n - 1 - k;
        q = kq == 0 ? 0 : ((kq - 1 + round) % (n - 1)) + 1;
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
      }
      double al = 0.0, be = 0.0, ga = 0.0;
      if (k < npair && q < M) {
        const double* ap = a.Zt + (int64_t)p * nc;
        const double* aq = a.Zt + (int64_t)q * nc;
        for (int64_t r = gl; r < nc; r += G) {
          const double u = ap[r], v = aq[r];
          al += u * u;
          be += v * v;
          ga += u * v;
        }
      }
      gsum[tid][0] = al;
      gsum[tid][1] = be;
      gsum[tid][2] = ga;
      __syncthreads();
      for (int off = G / 2; off > 0; off >>= 1) {
        if (gl < off) {
          gsum[tid][0] += gsum[tid + off][0];
          gsum[tid][1] += gsum[tid + off][1];
          gsum[tid][2] += gsum[tid + off][2];
        }
        __syncthreads();
      }
      if (gl == 0 && k < npair) {
        double c = 1.0, sn = 0.0;
        const double A0 = gsum[tid][0], B0 = gsum[tid][1], C0 = gsum[tid][2];
        if (q < M && C0 != 0.0 && fabs(C0) > 1e-15 * sqrt(A0 * B0)) {
          const double zeta = (B0 - A0) / (2.0 * C0);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = t * c;
          any_rot = 1;
        }
        pr_p[k] = p;
        pr_q[k] = q;
        cs_c[k] = c;
        cs_s[k] = sn;
      }
      __syncthreads();
      // rotate columns p, q of A and of E
      const int64_t span = nc + M;
      for (int64_t e = tid; e < (int64_t)npair * span; e += nt) {
        const int kk = (int)(e / span);
        const int64_t r = e - (int64_t)kk * span;
        if (cs_s[kk] == 0.0) continue;
        const int pp = pr_p[kk], qq = pr_q[kk];
        const double c = cs_c[kk], sn = cs_s[kk];
        if (r < nc) {
          double* ap = a.Zt + (int64_t)pp * nc;
          double* aq = a.Zt + (int64_t)qq * nc;
          const double u = ap[r], v = aq[r];
          ap[r] = c * u - sn * v;
          aq[r] = sn * u + c * v;
        } else {
          const int i = (int)(r - nc);
          double* ei = a.E + (int64_t)i * M;
          const double u = ei[pp], v = ei[qq];
          ei[pp] = c * u - sn * v;
          ei[qq] = sn * u + c * v;
        }
      }
      __syncthreads();
    }
    if (!any_rot) break;
  }

  // ---- Xi: singular vectors of the r_hat largest singular values ---------
  double* sig = a.R;  // squared column norms of the rotated A
  for (int i = tid; i < M; i += nt) {
    const double* ai = a.Zt + (int64_t)i * nc;
    double acc = 0.0;
    for (int64_t r = 0; r < nc; ++r) acc += ai[r] * ai[r];
    sig[i] = acc;
  }
  __syncthreads();
  for (int i = tid; i < M; i += nt) {
    const double li = sig[i];
    int rk = 0;
    for (int j = 0; j < M; ++j) {
      const double lj = sig[j];
      rk += (lj > li) || (lj == li && j < i);
    }
    a.rank[i] = rk;
  }
  __syncthreads();
  for (int e = tid; e < M * M; e += nt) {
    const int i = e / M, col = e % M;
    const int rk = a.rank[col];
    if (rk < rh) a.Xi[(int64_t)i * rh + rk] = a.E[(int64_t)i * M + col];
  }
  __syncthreads();

  // ---- Q-DEIM: column-pivoted QR of Xi^T (Drmac & Gugercin 2016) ----------
  // The rows of Xi are the columns of Xi^T.  Step j takes the row of largest
  // remaining norm (ties to the smallest index) and removes its direction
  // from every row (modified Gram-Schmidt); the picks are the first r_hat
  // pivots of the pivoted QR.  E (no longer needed) holds the rows.
  if (a.qdeim) {
    double* W = a.E;      // [M][rh]
    double* nrm = a.R;    // [M]
    double* qv = a.A;     // [rh]
    for (int e = tid; e < M * rh; e += nt) W[e] = a.Xi[e];
    for (int i = tid; i < M; i += nt) a.rank[i] = 0;  // 1 once picked
    __syncthreads();
    for (int j = 0; j < rh; ++j) {
      for (int i = tid; i < M; i += nt) {
        double acc = 0.0;
        for (int k = 0; k < rh; ++k) acc += W[(int64_t)i * rh + k] * W[(int64_t)i * rh + k];
        nrm[i] = a.rank[i] ? 0.0 : acc;
      }
      __syncthreads();
      const int pj = wg_argmax_abs(nrm, M, 1, sh);
      if (nrm[pj] <= 0.0) {
        if (tid == 0) *a.status = 1;
        return;
      }
      const double inv = 1.0 / sqrt(nrm[pj]);
      for (int k = tid; k < rh; k += nt) qv[k] = W[(int64_t)pj * rh + k] * inv;
      if (tid == 0) {
        a.P[j] = pj;
        a.rank[pj] = 1;
      }
      __syncthreads();
      for (int i = tid; i < M; i += nt) {
        double d = 0.0;
        for (int k = 0; k < rh; ++k) d += W[(int64_t)i * rh + k] * qv[k];
        for (int k = 0; k < rh; ++k) W[(int64_t)i * rh + k] -= d * qv[k];
      }
      __syncthreads();
    }
  }

  // ---- DEIM greedy -------------------------------------------------------
  double* res = a.R;
  for (int j = 0; j < rh && !a.qdeim; ++j) {
    if (j == 0) {
      for (int i = tid; i < M; i += nt) res[i] = a.Xi[(int64_t)i * rh];
      __syncthreads();
    } else {
      // A c = Xi[P, j] with A = Xi[P, :j]; the right-hand side sits in the
      // last row of the scratch, which the j x j system (j < rh) never uses
      double* Ac = a.A;
      double* cvec = a.A + (int64_t)rh * rh - rh;
      for (int e = tid; e < j * j; e += nt) {
        const int r = e / j, c = e % j;
        Ac[(int64_t)r * rh + c] = a.Xi[(int64_t)a.P[r] * rh + c];
      }
      for (int r = tid; r < j; r += nt) cvec[r] = a.Xi[(int64_t)a.P[r] * rh + j];
      __syncthreads();
      if (!wg_solve(Ac, j, rh, cvec, 1, 1, sh)) {
        if (tid == 0) *a.status = 1;
        return;
      }
      for (int i = tid; i < M; i += nt) {
        double acc = a.Xi[(int64_t)i * rh + j];
        for (int k = 0; k < j; ++k) acc -= a.Xi[(int64_t)i * rh + k] * cvec[k];
        res[i] = acc;
      }
      __syncthreads();
    }
    const int pj = wg_argmax_abs(res, M, 1, sh);
    if (tid == 0) a.P[j] = pj;
    __syncthreads();
  }

  // ---- reduced operators -------------------------------------------------
  for (int e = tid; e < rh * a.rl; e += nt) {
    const int i = e / a.rl, k = e % a.rl;
    a.Uh[e] = a.U[(int64_t)a.P[i] * a.rl + k];
  }
  for (int i = tid; i < rh; i += nt) a.bh[i] = a.b[a.P[i]];
  // V_hat = (P^T Xi)^{-T} Xi^T V^{l+1}: solve (P^T Xi)^T X = Xi^T V^{l+1}
  double* At = a.A;
  double* Bx = a.R;  // [rh][ro]
  for (int e = tid; e < rh * rh; e += nt) {
    const int r = e / rh, c = e % rh;
    At[(int64_t)r * rh + c] = a.Xi[(int64_t)a.P[c] * rh + r];
  }
  for (int e = tid; e < rh * a.ro; e += nt) {
    const int r = e / a.ro, c = e % a.ro;
    double acc = 0.0;
    for (int i = 0; i < M; ++i) acc += a.Xi[(int64_t)i * rh + r] * (double)a.Vn[(int64_t)i * a.ro + c];
    Bx[e] = acc;
  }
  __syncthreads();
  if (!wg_solve(At, rh, rh, Bx, a.ro, a.ro, sh)) {
    if (tid == 0) *a.status = 1;
    return;
  }
  for (int e = tid; e < rh * a.ro; e += nt) a.Vh[e] = (float)Bx[e];
}

}  // namespace lrnr

using namespace lrnr;

namespace {

template <class T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T) + 16);
}

}  // namespace

namespace {

int32_t build(const lrnr_net* net, const float* s_snap, int32_t n_s, const float* xt_snap,
              int64_t n_snap, const int32_t* r_hat, int32_t selection, fastlrnr_handle** out,
              void* stream) {
  if (!net || !s_snap || !xt_snap || !r_hat || !out) return LRNR_EINVAL;
  if (selection != LRNR_SEL_DEIM && selection != LRNR_SEL_QDEIM) return LRNR_EINVAL;
  *out = nullptr;
  const int L = net->L;
  if (L < 2 || L > LRNR_MAX_LAYERS || net->M[0] != 2 || net->M[L] != 1) return LRNR_EINVAL;
  if (n_s < 1 || n_snap < 1) return LRNR_EINVAL;
  if (!net->U || !net->V || !net->b) return LRNR_EINVAL;
  const int64_t ncols = (int64_t)n_s * n_snap;
  if (ncols > ((int64_t)1 << 24)) return LRNR_EUNSUPPORTED;
  KNet k{};
  k.L = L;
  int oU = 0, oV = 0, oB = 0, oS = 0;
  for (int l = 0; l <= L; ++l) k.M[l] = net->M[l];
  for (int l = 1; l <= L; ++l) {
    const int rl = net->r[l];
    if (l < L && (net->M[l] < 1 || net->M[l] > LRNR_MAX_WIDTH)) return LRNR_EUNSUPPORTED;
    if (rl < 1 || (l == 1 && rl > net->M[0]) || (l == L && rl > net->M[L])) return LRNR_EINVAL;
    if (rl > LRNR_MAX_RANK) return LRNR_EUNSUPPORTED;
    k.r[l] = rl;
    k.offU[l] = oU;
    k.offV[l] = oV;
    k.offB[l] = oB;
    k.offS[l] = oS;
    oU += net->M[l] * rl;
    oV += net->M[l - 1] * rl;
    oB += net->M[l];
    oS += rl;
  }
  k.r_total = oS;
  k.b_total = oB;
  k.U = net->U;
  k.V = net->V;
  k.b = net->b;
  for (int l = 1; l <= L - 1; ++l) {
    const int rh = r_hat[l - 1];
    if (rh < 1 || rh > net->M[l] || (int64_t)rh > ncols) return LRNR_EINVAL;
  }

  hipStream_t hs = static_cast<hipStream_t>(stream);
  auto* h = new fastlrnr_handle();
  lrnr_net& rn = h->net;
  rn.L = L;
  rn.M[0] = 2;
  rn.M[L] = 1;
  for (int l = 1; l <= L - 1; ++l) rn.M[l] = r_hat[l - 1];
  for (int l = 1; l <= L; ++l) rn.r[l] = net->r[l];
  size_t nU = 0, nV = 0, nb = 0, nP = 0, zsz = 0;
  int Mmax = 1;
  for (int l = 1; l <= L; ++l) {
    nU += (size_t)rn.M[l] * rn.r[l];
    nV += (size_t)rn.M[l - 1] * rn.r[l];
    nb += rn.M[l];
    if (l < L) {
      nP += r_hat[l - 1];
      zsz += (size_t)ncols * net->M[l];
      Mmax = std::max(Mmax, net->M[l]);
    }
  }
  double* Z = nullptr;
  double *E = nullptr, *Xi = nullptr, *A = nullptr, *R = nullptr;
  int *rank = nullptr, *Pd = nullptr, *status = nullptr;
  int32_t rc = LRNR_OK;
  hipError_t e = hipSuccess;
  const size_t Rn = std::max((size_t)Mmax, (size_t)Mmax * LRNR_MAX_RANK);
#define TRY(x)                 \
  do {                         \
    e = (x);                   \
    if (e != hipSuccess) {     \
      rc = LRNR_EHIP;          \
      goto done;               \
    }                          \
  } while (0)
  TRY(dalloc(&h->U, nU));
  TRY(dalloc(&h->V, nV));
  TRY(dalloc(&h->b, nb));
  TRY(dalloc(&Z, zsz));
  TRY(dalloc(&E, (size_t)Mmax * Mmax));
  TRY(dalloc(&Xi, (size_t)Mmax * Mmax));
  TRY(dalloc(&A, (size_t)Mmax * Mmax + Mmax));
  TRY(dalloc(&R, Rn));
  TRY(dalloc(&rank, (size_t)Mmax));
  TRY(dalloc(&Pd, nP));
  TRY(dalloc(&status, 1));
  TRY(hipMemsetAsync(status, 0, sizeof(int), hs));
  {
    const int bx = 128;
    hipLaunchKernelGGL(snapshot_kernel, dim3((unsigned)((ncols + bx - 1) / bx)), dim3(bx), 0, hs,
                       k, s_snap, n_s, xt_snap, n_snap, Z, ncols);
    TRY(hipGetLastError());
    size_t zoff = 0, uoff = 0, voff = (size_t)2 * rn.r[1], boff = 0, poff = 0;
    for (int l = 1; l <= L - 1; ++l) {
      const int M = net->M[l], rh = r_hat[l - 1];
      SelArgs sa{};
      sa.M = M;
      sa.r_hat = rh;
      sa.rl = net->r[l];
      sa.ro = net->r[l + 1];
      sa.Zt = Z + zoff;
      sa.ncols = ncols;
      sa.E = E;
      sa.Xi = Xi;
      sa.A = A;
      sa.R = R;
      sa.rank = rank;
      sa.P = Pd + poff;
      sa.U = net->U + k.offU[l];
      sa.b = net->b + k.offB[l];
      sa.Vn = net->V + k.offV[l + 1];
      sa.Uh = h->U + uoff;
      sa.bh = h->b + boff;
      sa.Vh = h->V + voff;
      sa.status = status;
      sa.qdeim = selection == LRNR_SEL_QDEIM;
      hipLaunchKernelGGL(select_kernel, dim3(1), dim3(kSelThreads), 0, hs, sa);
      TRY(hipGetLastError());
      zoff += (size_t)ncols * M;
      uoff += (size_t)rh * net->r[l];
      boff += rh;
      voff += (size_t)rh * net->r[l + 1];
      poff += rh;
    }
    // unchanged parts: V^1 (input layer), U^L and b^L (output layer)
    TRY(hipMemcpyAsync(h->V, net->V, sizeof(float) * 2 * net->r[1], hipMemcpyDeviceToDevice, hs));
    TRY(hipMemcpyAsync(h->U + uoff, net->U + k.offU[L], sizeof(float) * net->r[L],
                       hipMemcpyDeviceToDevice, hs));
    TRY(hipMemcpyAsync(h->b + boff, net->b + k.offB[L], sizeof(float), hipMemcpyDeviceToDevice,
                       hs));
    h->P.resize(nP);
    int st = 0;
    TRY(hipMemcpyAsync(h->P.data(), Pd, nP * sizeof(int32_t), hipMemcpyDeviceToHost, hs));
    TRY(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, hs));
    TRY(hipStreamSynchronize(hs));
    if (st) rc = LRNR_ESINGULAR;
  }
done:
#undef TRY
  if (e != hipSuccess) set_status_detail(hipGetErrorString(e));
  if (rc == LRNR_ESINGULAR)
    set_status_detail("zero pivot in the DEIM or V_hat system, or no row left for Q-DEIM");
  (void)hipFree(Z);
  (void)hipFree(E);
  (void)hipFree(Xi);
  (void)hipFree(A);
  (void)hipFree(R);
  (void)hipFree(rank);
  (void)hipFree(status);
  h->Pd = Pd;
  if (rc != LRNR_OK) {
    fastlrnr_destroy(h);
    return rc;
  }
  rn.U = h->U;
  rn.V = h->V;
  rn.b = h->b;
  *out = h;
  return LRNR_OK;
}

}  // namespace

extern "C" {

int32_t fastlrnr_build(const lrnr_net* net, const float* s_snap, int32_t n_s,
                       const float* xt_snap, int64_t n_snap, const int32_t* r_hat,
                       fastlrnr_handle** out, void* stream) {
  return build(net, s_snap, n_s, xt_snap, n_snap, r_hat, LRNR_SEL_DEIM, out, stream);
}

int32_t fastlrnr_build_sel(const lrnr_net* net, const float* s_snap, int32_t n_s,
                           const float* xt_snap, int64_t n_snap, const int32_t* r_hat,
                           int32_t selection, fastlrnr_handle** out, void* stream) {
  return build(net, s_snap, n_s, xt_snap, n_snap, r_hat, selection, out, stream);
}

int32_t fastlrnr_get_net(const fastlrnr_handle* h, lrnr_net* out) {
  if (!h || !out) return LRNR_EINVAL;
  *out = h->net;
  return LRNR_OK;
}

int32_t fastlrnr_get_indices(const fastlrnr_handle* h, int32_t* P) {
  if (!h || !P) return LRNR_EINVAL;
  std::memcpy(P, h->P.data(), h->P.size() * sizeof(int32_t));
  return LRNR_OK;
}

int32_t fastlrnr_grad_s(const fastlrnr_handle* h, const float* s, const float* mu,
                        const lrnr_points* pts, const lrnr_loss_cfg* cfg, float* grad_s,
                        float* loss, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return LRNR_EINVAL;
  return lrnr_grad_s(&h->net, s, mu, pts, cfg, grad_s, nullptr, loss, ws, ws_bytes, stream);
}

int32_t fastlrnr_bias_basis(const fastlrnr_handle* h, const lrnr_bias_basis* full, float* B_hat,
                            lrnr_bias_basis* reduced, void* stream) {
  if (!h) return fail(LRNR_EINVAL, "NULL handle");
  return bias_gather(full, h->P.data(), h->Pd, &h->net, B_hat, reduced,
                     static_cast<hipStream_t>(stream));
}

int32_t fastlrnr_destroy(fastlrnr_handle* h) {
  if (!h) return LRNR_EINVAL;
  (void)hipFree(h->U);
  (void)hipFree(h->V);
  (void)hipFree(h->b);
  (void)hipFree(h->Pd);
  delete h;
  return LRNR_OK;
}

}  // extern "C"

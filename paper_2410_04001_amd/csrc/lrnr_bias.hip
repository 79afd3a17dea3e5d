// Factored biases b^l = B^l s_b^l (the treatment of the biases like the
// weights that Section 2.1 mentions): composition of the biases from their
// coefficients before a step, the chain rule grad_sb^l = B^lT grad_b^l after
// it, and the row gather that gives a FastLRNR its reduced basis (eq. 2.7
// applied to b = B s_b).  All three are small: one workgroup per layer, sums
// in FP64 in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lrnr_bias.h"

namespace lrnr {
namespace {

constexpr int kBiasThreads = 256;

struct KBias {
  int L;
  int M[LRNR_MAX_LAYERS + 1];
  int q[LRNR_MAX_LAYERS + 1];
  int64_t offB[LRNR_MAX_LAYERS + 1];   // float offset of B^l
  int offS[LRNR_MAX_LAYERS + 1];       // offset of s_b^l
  int offb[LRNR_MAX_LAYERS + 1];       // offset of b^l
  const float* B;
};

// b^l[i] = sum_j B^l[i][j] s_b^l[j], j ascending
__global__ void __launch_bounds__(kBiasThreads) bias_compose_kernel(KBias k, const float* sb,
                                                                    float* b) {
  const int l = blockIdx.x + 1, M = k.M[l], q = k.q[l];
  const float* B = k.B + k.offB[l];
  const float* s = sb + k.offS[l];
  for (int i = threadIdx.x; i < M; i += kBiasThreads) {
    double acc = 0.0;
    for (int j = 0; j < q; ++j) acc += (double)B[(int64_t)i * q + j] * (double)s[j];
    b[k.offb[l] + i] = (float)acc;
  }
}

// grad_sb^l[j] = sum_i B^l[i][j] grad_b^l[i], i ascending
__global__ void __launch_bounds__(kBiasThreads) bias_grad_kernel(KBias k, const float* gb,
                                                                 float* gsb) {
  const int l = blockIdx.x + 1, M = k.M[l], q = k.q[l];
  const float* B = k.B + k.offB[l];
  const float* g = gb + k.offb[l];
  for (int j = threadIdx.x; j < q; j += kBiasThreads) {
    // loads issued eight rows at a time, added in row order
    double acc = 0.0;
    int i = 0;
    for (; i + 8 <= M; i += 8) {
      float bv[8], gv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        bv[u] = B[(int64_t)(i + u) * q + j];
        gv[u] = g[i + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += (double)bv[u] * (double)gv[u];
    }
    for (; i < M; ++i) acc += (double)B[(int64_t)i * q + j] * (double)g[i];
    gsb[k.offS[l] + j] = (float)acc;
  }
}

struct KGather {
  int L;
  int rows[LRNR_MAX_LAYERS + 1];       // rows of the reduced basis
  int q[LRNR_MAX_LAYERS + 1];
  int64_t offF[LRNR_MAX_LAYERS + 1];   // B^l in the full basis
  int64_t offR[LRNR_MAX_LAYERS + 1];   // B_hat^l in the reduced basis
  int offP[LRNR_MAX_LAYERS + 1];       // P^l in the concatenated indices
  const int32_t* P;                    // hidden layers 1..L-1
  const float* Bf;
  float* Br;
};

// B_hat^l[i][:] = B^l[P^l[i]][:] for hidden layers; the output layer's rows as they are
__global__ void __launch_bounds__(kBiasThreads) bias_gather_kernel(KGather g) {
  const int l = blockIdx.x + 1, q = g.q[l], n = g.rows[l] * q;
  for (int e = threadIdx.x; e < n; e += kBiasThreads) {
    const int i = e / q, j = e - i * q;
    const int src = (l < g.L) ? g.P[g.offP[l] + i] : i;
    g.Br[g.offR[l] + e] = g.Bf[g.offF[l] + (int64_t)src * q + j];
  }
}

int32_t make_kbias(const lrnr_bias_basis* bb, KBias* k) {
  if (!bb) return fail(LRNR_EINVAL, "NULL bias basis");
  if (bb->L < 1 || bb->L > LRNR_MAX_LAYERS) return fail(LRNR_EINVAL, "bias basis L=%d", bb->L);
  k->L = bb->L;
  int64_t oB = 0;
  int oS = 0, ob = 0;
  for (int l = 1; l <= bb->L; ++l) {
    const int M = bb->M[l], q = bb->q[l];
    if (M < 1 || M > LRNR_MAX_WIDTH) return fail(LRNR_EINVAL, "bias basis M[%d]=%d", l, M);
    if (q < 0 || q > LRNR_MAX_RANK) return fail(LRNR_EINVAL, "bias basis q[%d]=%d", l, q);
    k->M[l] = M;
    k->q[l] = q;
    k->offB[l] = oB;
    k->offS[l] = oS;
    k->offb[l] = ob;
    oB += (int64_t)M * q;
    oS += q;
    ob += M;
  }
  if (oB > 0 && !bb->B) return fail(LRNR_EINVAL, "NULL bias basis B");
  k->B = bb->B;
  return LRNR_OK;
}

}  // namespace

int32_t bias_gather(const lrnr_bias_basis* full, const int32_t* P_host, const int32_t* P_dev,
                    const lrnr_net* reduced_net, float* B_hat, lrnr_bias_basis* reduced,
                    hipStream_t stream) {
  KBias kf;
  int32_t rc = make_kbias(full, &kf);
  if (rc != LRNR_OK) return rc;
  const int L = reduced_net->L;
  if (full->L != L) return fail(LRNR_EINVAL, "bias basis L=%d, FastLRNR L=%d", full->L, L);
  if (full->M[L] != reduced_net->M[L])
    return fail(LRNR_EINVAL, "bias basis M[L]=%d, net M[L]=%d", full->M[L], reduced_net->M[L]);
  KGather g{};
  g.L = L;
  int64_t oR = 0;
  int oP = 0;
  for (int l = 1; l <= L; ++l) {
    g.rows[l] = reduced_net->M[l];
    g.q[l] = kf.q[l];
    g.offF[l] = kf.offB[l];
    g.offR[l] = oR;
    g.offP[l] = oP;
    if (l < L) {
      for (int i = 0; i < g.rows[l]; ++i)
        if (P_host[oP + i] < 0 || P_host[oP + i] >= full->M[l])
          return fail(LRNR_EINVAL, "index %d of layer %d outside the basis rows (%d)",
                      P_host[oP + i], l, full->M[l]);
      oP += g.rows[l];
    }
    oR += (int64_t)g.rows[l] * g.q[l];
  }
  if (oR > 0 && !B_hat) return fail(LRNR_EINVAL, "NULL B_hat");
  g.P = P_dev;
  g.Bf = full->B;
  g.Br = B_hat;
  if (reduced) {
    reduced->L = L;
    reduced->M[0] = full->M[0];
    reduced->q[0] = 0;
    for (int l = 1; l <= L; ++l) {
      reduced->M[l] = g.rows[l];
      reduced->q[l] = g.q[l];
    }
    for (int l = L + 1; l <= LRNR_MAX_LAYERS; ++l) reduced->M[l] = reduced->q[l] = 0;
    reduced->B = B_hat;
  }
  if (oR == 0) return LRNR_OK;
  hipLaunchKernelGGL(bias_gather_kernel, dim3(L), dim3(kBiasThreads), 0, stream, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "bias gather launch");
  return LRNR_OK;
}

}  // namespace lrnr

using namespace lrnr;

extern "C" {

int32_t lrnr_bias_compose(const lrnr_bias_basis* bb, const float* s_b, float* b, void* stream) {
  KBias k;
  int32_t rc = make_kbias(bb, &k);
  if (rc != LRNR_OK) return rc;
  if (!b) return fail(LRNR_EINVAL, "NULL b");
  if (k.offS[k.L] + k.q[k.L] > 0 && !s_b) return fail(LRNR_EINVAL, "NULL s_b");
  hipLaunchKernelGGL(bias_compose_kernel, dim3(k.L), dim3(kBiasThreads), 0,
                     static_cast<hipStream_t>(stream), k, s_b, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "bias compose launch");
  return LRNR_OK;
}

int32_t lrnr_bias_grad(const lrnr_bias_basis* bb, const float* grad_b, float* grad_sb,
                       void* stream) {
  KBias k;
  int32_t rc = make_kbias(bb, &k);
  if (rc != LRNR_OK) return rc;
  if (k.offS[k.L] + k.q[k.L] == 0) return LRNR_OK;
  if (!grad_b || !grad_sb) return fail(LRNR_EINVAL, "NULL grad_b or grad_sb");
  hipLaunchKernelGGL(bias_grad_kernel, dim3(k.L), dim3(kBiasThreads), 0,
                     static_cast<hipStream_t>(stream), k, grad_b, grad_sb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "bias grad launch");
  return LRNR_OK;
}

}  // extern "C"

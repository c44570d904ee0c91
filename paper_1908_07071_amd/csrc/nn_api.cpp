// C ABI of the learned patch correction: network buffers, forward and
// backward passes, Adam steps, training data from the method's own patch
// V-cycles, and the network in place of the patch V-cycles of eq. as.
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "lor_handle.h"

struct lor_nn {
  lor_handle *h = nullptr;
  int C = 32, G = 0, G3 = 0, maxb = 0;
  int cin[3] = {}, cout[3] = {}, K27[3] = {}, Kp[3] = {}, Np[3] = {};
  int64_t off[3] = {};  // offset of each layer in the flat parameters
  int64_t nparam = 0, npad_max = 0;
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint16_t *Wb[3] = {};
  uint16_t *Wf[3] = {};  // fused path: weights in MFMA fragment order
  float *bias[3] = {};
  uint16_t *a[3] = {};  // layer inputs (bf16)
  float *z[3] = {};     // pre-activations [npad][Np]
  uint16_t *cols = nullptr, *dz16 = nullptr;
  float *dcols = nullptr, *dz = nullptr, *dW = nullptr, *y = nullptr, *Xbuf = nullptr;
  double *part = nullptr, *sbuf = nullptr;
  double *scal = nullptr;   // device scalars of a training step: mask count, loss sum
  float *yall = nullptr;    // warm start: predictions of every patch [J][G^3]
  double *sall = nullptr;   // and their scales [J]
  int step = 0;
  bool fused = false;  // fused convolution kernels for this shape
  std::vector<void *> allocs;
  template <class T>
  hipError_t alloc(T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count * sizeof(T), 16));
    if (e != hipSuccess) return e;
    allocs.push_back(q);
    *p = static_cast<T *>(q);
    return hipSuccess;
  }
  ~lor_nn() {
    for (void *p : allocs) (void)hipFree(p);
  }
};

namespace {

#define NCHK(x)                                 \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return LOR_EHIP;      \
  } while (0)

inline int64_t pad16(int64_t x) { return (x + 15) / 16 * 16; }

int64_t param_count(int C) {
  return int64_t(27) * 2 * C + C + int64_t(27) * C * C + C + int64_t(27) * C + 1;
}

int pack_all(lor_nn *nn, hipStream_t st) {
  for (int l = 0; l < 3; ++l) {
    NCHK(nn_pack(nn->w + nn->off[l], nn->K27[l], nn->cout[l], nn->Kp[l], nn->Np[l], nn->Wb[l],
                 nn->bias[l], st));
    if (nn->fused) NCHK(nn_conv_frag(nn->Wb[l], nn->Kp[l], nn->Np[l], nn->Wf[l], st));
  }
  return LOR_OK;
}

// Forward pass of nb samples X [nb][G^3][2]; output in nn->y.
// Network output y for nb patches.  keep: also the pre-activations z[l]
// (the backward pass needs them).  The fused convolution kernels serve the
// supported shapes, the explicit im2col + GEMM path the others.
int forward(lor_nn *nn, const float *X, int nb, const double *flag, hipStream_t st, bool keep = true,
            float *yout = nullptr) {
  const int64_t rows = int64_t(nb) * nn->G3, npad = pad16(rows);
  NCHK(nn_input(X, rows, npad, nn->a[0], flag, st));
  if (nn->fused) {
    float *y = yout ? yout : nn->y;
    for (int l = 0; l < 3; ++l)
      NCHK(nn_conv_layer(nn->C, l, nn->a[l], nb, nn->G, nn->Wf[l], nn->bias[l], keep ? nn->z[l] : nullptr,
                         l < 2 ? nn->a[l + 1] : nullptr, X, l == 2 ? y : nullptr, flag, st));
    return LOR_OK;
  }
  for (int l = 0; l < 3; ++l) {
    NCHK(nn_im2col(nn->a[l], rows, nn->G, nn->cin[l], nn->Kp[l], npad, nn->cols, flag, st));
    NCHK(nn_gemm(int(npad), nn->Np[l], nn->Kp[l], nn->cols, nn->Kp[l], 1, nn->Wb[l], nn->Np[l], 1,
                 nn->z[l], nn->Np[l], false, st));
    NCHK(nn_bias_relu(nn->z[l], rows, nn->cout[l], nn->Np[l], nn->bias[l], l < 2 ? nn->a[l + 1] : nullptr,
                      flag, st));
  }
  NCHK(nn_output(nn->z[2], nn->Np[2], X, rows, yout ? yout : nn->y, flag, st));
  return LOR_OK;
}

// Loss of the batch and the flat float32 gradient in nn->g.  Every
// reduction (mask count, loss, bias gradients) is finished on the device, in
// double over per-block partials in block order; the host waits once, for the
// mask count and the loss.
int backward(lor_nn *nn, const float *X, const float *T, int nb, double *loss, hipStream_t st) {
  const int64_t rows = int64_t(nb) * nn->G3, npad = pad16(rows);
  int rc = forward(nn, X, nb, nullptr, st);
  if (rc != LOR_OK) return rc;
  // number of masked points -> scal[0]
  NCHK(nn_colsum(X, rows, 2, 1, 1, nn->part, st));
  NCHK(nn_sum_partials(nn->part, nn_red_blocks(rows), 1, nn->scal, nullptr, st));
  NCHK(nn_loss(nn->y, T, X, rows, npad, nn->Np[2], nn->scal, nn->dz, nn->dz16, nn->part, st));
  NCHK(nn_sum_partials(nn->part, nn_red_blocks(npad), 1, nn->scal + 1, nullptr, st));
  for (int l = 2; l >= 0; --l) {
    const int Np = nn->Np[l], Kp = nn->Kp[l], cout = nn->cout[l];
    // dW = cols^T dz (sum over all rows), db = column sums of dz
    NCHK(nn_im2col(nn->a[l], rows, nn->G, nn->cin[l], Kp, npad, nn->cols, nullptr, st));
    NCHK(nn_gemm(Kp, Np, int(npad), nn->cols, 1, Kp, nn->dz16, Np, 1, nn->dW, Np, false, st));
    NCHK(nn_grad_gather(nn->dW, nn->K27[l], cout, Np, nn->g + nn->off[l], st));
    NCHK(nn_colsum(nn->dz, rows, Np, 0, cout, nn->part, st));
    NCHK(nn_sum_partials(nn->part, nn_red_blocks(rows), cout, nullptr,
                         nn->g + nn->off[l] + int64_t(nn->K27[l]) * cout, st));
    if (l > 0) {
      // input gradient: dcols = dz W^T, then col2im and the ReLU of layer l-1
      NCHK(nn_gemm(int(npad), Kp, Np, nn->dz16, Np, 1, nn->Wb[l], 1, Np, nn->dcols, Kp, false, st));
      NCHK(nn_col2im_relu(nn->dcols, rows, npad, nn->G, nn->cin[l], Kp, nn->z[l - 1], nn->Np[l - 1],
                          nn->dz, nn->dz16, st));
    }
  }
  double hs[2];
  NCHK(hipMemcpyAsync(hs, nn->scal, sizeof(hs), hipMemcpyDeviceToHost, st));
  NCHK(hipStreamSynchronize(st));
  // no masked point: the gradient is not defined (and not applied)
  if (!(hs[0] > 0.0)) return LOR_EINVAL;
  if (loss) *loss = hs[1] / hs[0];
  return LOR_OK;
}

}  // namespace

int nn_apply_patches(lor_nn *nn, const double *r, double *z, const double *flag, hipStream_t st) {
  const int J = nn->h->J;
  for (int first = 0; first < J; first += nn->maxb) {
    const int cnt = std::min(nn->maxb, J - first);
    NCHK(nn_gather(nn->h->md, first, cnt, r, nn->Xbuf, nn->sbuf, flag, st));
    int rc = forward(nn, nn->Xbuf, cnt, flag, st, false);
    if (rc != LOR_OK) return rc;
    NCHK(nn_scatter(nn->h->md, first, cnt, nn->y, nn->sbuf, z, flag, st));
  }
  return LOR_OK;
}

// Warm start: per chunk of patches, the network's prediction y_j (scaled by
// s_j) starts the patch V-cycle, which adds y_j + V_j(r_j - A_j y_j) into z.
int nn_apply_patches_warm(lor_nn *nn, const double *r, double *z, const double *flag,
                          hipStream_t st) {
  const int J = nn->h->J;
  if (!nn->yall || !nn->sall) return LOR_ESTATE;  // allocated when attached for a warm start
  for (int first = 0; first < J; first += nn->maxb) {
    const int cnt = std::min(nn->maxb, J - first);
    NCHK(nn_gather(nn->h->md, first, cnt, r, nn->Xbuf, nn->sall + first, flag, st));
    int rc = forward(nn, nn->Xbuf, cnt, flag, st, false, nn->yall + size_t(first) * nn->G3);
    if (rc != LOR_OK) return rc;
  }
  NCHK(launch_patch_vcycle_warm(nn->h->pa, 0, J, r, z, nn->yall, nn->sall, flag, st));
  return LOR_OK;
}

extern "C" {

int lor_nn_param_count(int channels, int64_t *count) {
  if (!count || channels < 16 || channels > 64 || channels % 16) return LOR_EINVAL;
  *count = param_count(channels);
  return LOR_OK;
}

int lor_nn_create(lor_handle_t *h, int channels, const double *params, int max_batch, void *stream,
                  lor_nn_t **out) {
  if (!out) return LOR_EINVAL;
  *out = nullptr;
  if (!h || !params || channels < 16 || channels > 64 || channels % 16 || max_batch < 1)
    return LOR_EINVAL;
  if (h->dim != 3 || h->method != LOR_CG || !h->has_prec) return LOR_ESTATE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::unique_ptr<lor_nn> nn(new (std::nothrow) lor_nn());
  if (!nn) return LOR_ENOMEM;
  nn->h = h;
  nn->C = channels;
  nn->G = 2 * h->p - 1;
  nn->G3 = nn->G * nn->G * nn->G;
  nn->maxb = max_batch;
  nn->fused = nn_conv_supported(channels, nn->G);
  if (nn->fused) NCHK(nn_conv_prepare(channels));
  const int C = channels;
  const int cin[3] = {2, C, C}, cout[3] = {C, C, 1};
  int64_t o = 0;
  int Kmax = 0, Npmax = 0;
  for (int l = 0; l < 3; ++l) {
    nn->cin[l] = cin[l];
    nn->cout[l] = cout[l];
    nn->K27[l] = 27 * cin[l];
    nn->Kp[l] = int(pad16(nn->K27[l]));
    nn->Np[l] = int(pad16(cout[l]));
    nn->off[l] = o;
    o += int64_t(nn->K27[l]) * cout[l] + cout[l];
    Kmax = std::max(Kmax, nn->Kp[l]);
    Npmax = std::max(Npmax, nn->Np[l]);
  }
  nn->nparam = o;
  const int64_t npad = pad16(int64_t(max_batch) * nn->G3);
  nn->npad_max = npad;
  NCHK(nn->alloc(&nn->w, o));
  NCHK(nn->alloc(&nn->m, o));
  NCHK(nn->alloc(&nn->v, o));
  NCHK(nn->alloc(&nn->g, o));
  for (int l = 0; l < 3; ++l) {
    NCHK(nn->alloc(&nn->Wb[l], size_t(nn->Kp[l]) * nn->Np[l]));
    NCHK(nn->alloc(&nn->Wf[l], size_t(nn->Kp[l]) * nn->Np[l]));
    NCHK(nn->alloc(&nn->bias[l], nn->Np[l]));
    NCHK(nn->alloc(&nn->a[l], size_t(npad) * cin[l]));
    NCHK(nn->alloc(&nn->z[l], size_t(npad) * nn->Np[l]));
  }
  NCHK(nn->alloc(&nn->cols, size_t(npad) * Kmax));
  NCHK(nn->alloc(&nn->dcols, size_t(npad) * Kmax));
  NCHK(nn->alloc(&nn->dz, size_t(npad) * Npmax));
  NCHK(nn->alloc(&nn->dz16, size_t(npad) * Npmax));
  NCHK(nn->alloc(&nn->dW, size_t(Kmax) * Npmax));
  NCHK(nn->alloc(&nn->y, size_t(npad)));
  NCHK(nn->alloc(&nn->Xbuf, size_t(max_batch) * nn->G3 * 2));
  NCHK(nn->alloc(&nn->sbuf, size_t(max_batch)));
  NCHK(nn->alloc(&nn->part, size_t(Npmax) * kPartStride));
  NCHK(nn->alloc(&nn->scal, 2));
  std::vector<float> w32(o);
  for (int64_t i = 0; i < o; ++i) {
    if (!std::isfinite(params[i])) return LOR_EINVAL;
    w32[i] = float(params[i]);
  }
  NCHK(hipMemcpyAsync(nn->w, w32.data(), o * sizeof(float), hipMemcpyHostToDevice, st));
  NCHK(nn_fill(nn->m, o, 0.f, st));
  NCHK(nn_fill(nn->v, o, 0.f, st));
  NCHK(nn_fill(nn->dz, npad * Npmax, 0.f, st));
  int rc = pack_all(nn.get(), st);
  if (rc != LOR_OK) return rc;
  NCHK(hipStreamSynchronize(st));
  *out = nn.release();
  return LOR_OK;
}

int lor_nn_get_params(const lor_nn_t *nn, double *params) {
  if (!nn || !params) return LOR_EINVAL;
  std::vector<float> w32(nn->nparam);
  NCHK(hipMemcpy(w32.data(), nn->w, nn->nparam * sizeof(float), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < nn->nparam; ++i) params[i] = w32[i];
  return LOR_OK;
}

int lor_nn_shape(const lor_nn_t *nn, int *npatch, int *grid) {
  if (!nn || !npatch || !grid) return LOR_EINVAL;
  *npatch = nn->h->J;
  *grid = nn->G;
  return LOR_OK;
}

int lor_nn_patch_data(lor_nn_t *nn, const double *r, float *X, float *T, double *scale,
                      void *stream) {
  if (!nn || !r || !X || !T || !scale) return LOR_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  lor_handle *h = nn->h;
  NCHK(nn_gather(h->md, 0, h->J, r, X, scale, nullptr, st));
  NCHK(nn_fill(T, int64_t(h->J) * nn->G3, 0.f, st));
  NCHK(launch_patch_vcycle(h->pa, h->J, r, nullptr, nullptr, st, T, scale));
  return LOR_OK;
}

int lor_nn_forward(lor_nn_t *nn, const float *X, int nb, float *Y, void *stream) {
  if (!nn || !X || !Y || nb < 1 || nb > nn->maxb) return LOR_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = forward(nn, X, nb, nullptr, st);
  if (rc != LOR_OK) return rc;
  NCHK(hipMemcpyAsync(Y, nn->y, size_t(nb) * nn->G3 * sizeof(float), hipMemcpyDeviceToDevice, st));
  return LOR_OK;
}

int lor_nn_gradients(lor_nn_t *nn, const float *X, const float *T, int nb, double *loss,
                     double *grad, void *stream) {
  if (!nn || !X || !T || !grad || nb < 1 || nb > nn->maxb) return LOR_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = backward(nn, X, T, nb, loss, st);
  if (rc != LOR_OK) return rc;
  std::vector<float> g32(nn->nparam);
  NCHK(hipMemcpy(g32.data(), nn->g, nn->nparam * sizeof(float), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < nn->nparam; ++i) grad[i] = g32[i];
  return LOR_OK;
}

int lor_nn_train_step(lor_nn_t *nn, const float *X, const float *T, int nb, double lr,
                      double *loss, void *stream) {
  if (!nn || !X || !T || nb < 1 || nb > nn->maxb || !(lr > 0.0)) return LOR_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = backward(nn, X, T, nb, loss, st);
  if (rc != LOR_OK) return rc;
  const double b1 = 0.9, b2 = 0.999;
  ++nn->step;
  const double c1 = 1.0 / (1.0 - std::pow(b1, nn->step)), c2 = 1.0 / (1.0 - std::pow(b2, nn->step));
  NCHK(nn_adam(nn->w, nn->m, nn->v, nn->g, nn->nparam, float(lr), float(b1), float(b2), 1e-8f,
               float(c1), float(c2), st));
  return pack_all(nn, st);
}

int lor_nn_attach(lor_handle_t *h, lor_nn_t *nn, int mode) {
  if (!h || (mode != LOR_NN_OFF && mode != LOR_NN_REPLACE && mode != LOR_NN_WARMSTART))
    return LOR_EINVAL;
  if (mode != LOR_NN_OFF && (!nn || nn->h != h)) return LOR_EINVAL;
  if (mode != LOR_NN_OFF && (h->opt.patch_mode != LOR_PATCH_VERTEX || h->opt.deterministic))
    return LOR_ESTATE;
  // the network's own scatter adds corrections unweighted
  if (mode == LOR_NN_REPLACE && h->opt.prolong_weights != LOR_PROLONG_SUM) return LOR_ESTATE;
  if (mode == LOR_NN_WARMSTART && !nn->yall) {
    // predictions and scales of every patch, so that one launch runs all
    // the warm-started V-cycles
    if (nn->alloc(&nn->yall, size_t(h->J) * nn->G3) != hipSuccess ||
        nn->alloc(&nn->sall, size_t(h->J)) != hipSuccess)
      return LOR_ENOMEM;
  }
  h->nn = mode == LOR_NN_OFF ? nullptr : nn;
  h->nn_mode = mode;
  return LOR_OK;
}

int lor_nn_free(lor_nn_t *nn) {
  if (!nn) return LOR_EINVAL;
  if (nn->h && nn->h->nn == nn) {
    nn->h->nn = nullptr;
    nn->h->nn_mode = LOR_NN_OFF;
  }
  delete nn;
  return LOR_OK;
}

int lor_bf16_gemm(int M, int N, int K, const uint16_t *A, int64_t ai, int64_t ak, const uint16_t *B,
                  int64_t bk, int64_t bj, float *C, int64_t ldc, void *stream) {
  if (!A || !B || !C || M <= 0 || N <= 0 || K <= 0 || M % 16 || N % 16 || K % 16) return LOR_EINVAL;
  NCHK(nn_gemm(M, N, K, A, ai, ak, B, bk, bj, C, ldc, false, static_cast<hipStream_t>(stream)));
  return LOR_OK;
}

}  // extern "C"

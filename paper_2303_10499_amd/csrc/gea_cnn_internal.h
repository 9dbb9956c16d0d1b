// gea_cnn_internal.h -- the learned-preconditioner network inside the
// library: layer geometry, buffers carved from a workspace, and the host
// functions that enqueue its kernels (gea_cnn.hip).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "gea.h"
#include "gea_internal.h"

namespace gea {

typedef uint16_t bf16_t;  // bfloat16 bit pattern

constexpr int kCnnLayers = 6;
constexpr int kCnnInputs = 2;  // r/s, c/diag

struct CnnDims {
  int nx, ny, nz, npix;  // ny = 1 in 2D
};

struct CnnLayer {
  int cin, cout;      // logical channels
  int cin_p, cout_p;  // padded: inputs to a multiple of 8, outputs to a multiple of 16
  int level;          // resolution level (0 full, 1 half, 2 quarter)
  int kpad;           // row length of W: taps*cin_p rounded up to 32
  int kpad_t;         // row length of the flipped/transposed W (taps*cout_p rounded to 32)
  int cin_t_p;        // rows of the transposed W: cin padded to 16
  long woff, boff;    // offsets of W and b in the packed FP32 parameters
};

struct Cnn {
  int ndim = 2;
  bool train = false;
  hipStream_t s = nullptr;
  CnnDims d[3];
  CnnLayer L[kCnnLayers];
  long nparams = 0;
  int nsplit = 1;        // pixel splits of the weight-gradient reduction
  long part_floats = 0;  // size of that reduction's partial buffer
  // parameters
  float* master = nullptr;
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  bf16_t* W[kCnnLayers] = {};
  bf16_t* Wt[kCnnLayers] = {};
  bf16_t* W0 = nullptr;  // layer 0 weights in the (tap, 2 channels) K order
  bf16_t* W5 = nullptr;  // layer 5 weights transposed: [tap (32)][channel (16)]
  bf16_t* Wz[kCnnLayers] = {};  // 3D layers 1, 3, 4: weights packed for the z-march kernel
  bf16_t* W0z = nullptr;        // 3D layer 0: its three z-march B operands
  float* bias[kCnnLayers] = {};
  // forward activations (bf16, channels last)
  uint32_t* x2;  // input, 2 bf16 channels per cell (what layer 0 reads)
  bf16_t *xin, *e0, *p0, *e1, *p1, *e2, *c1, *d1, *c0, *d0;  // xin: input padded to 8 (training)
  float* y;   // output, 1 channel
  float* xf;  // FP32 staging of the 2-channel input
  // backward
  float *t, *dy5, *dd0, *dc0, *dd1, *de0, *dc1, *de2, *de1, *dp1, *dp0;
  bf16_t *q5, *q4, *q3, *q2, *q1, *q0;  // bf16 copies of the (masked) output gradients
  float* part;
  double* lpart;
};

long cnn_param_count(int ndim);
// Fills geometry and, with base != null, the pointers; returns the end offset.
size_t cnn_carve(Cnn& n, int ndim, int nx, int ny, int nz, bool train, char* base, size_t off);
bool cnn_dims_ok(int ndim, int nx, int ny, int nz);

void cnn_pack_weights(Cnn& n);                 // master -> bf16 W, Wt and bias
void cnn_input_from_f32(Cnn& n);              // xf (npix x 2 FP32) -> xin
void cnn_forward(Cnn& n);                      // xin -> y
void cnn_conv_layer(Cnn& n, int layer);        // the forward convolution of one layer
double cnn_layer_flops(const Cnn& n, int layer);  // its multiply-adds x 2 (logical channels)
void cnn_backward(Cnn& n, bool accumulate);    // t, last forward -> grad (loss partials in lpart)
void cnn_adam(Cnn& n, float lr, float scale, int step);
int cnn_loss_partials(const Cnn& n);           // number of loss partials in lpart

// Learned preconditioner support: xin from an FP32 residual r (scale 1/s
// from *inv_s on the device) and c/diag; out = s * y.
void cnn_input_from_residual(Cnn& n, const float* r, const double* inv_s, const float* c,
                             const float* dinv);
// inference only: the forward pass with the last layer writing out = (float)*s * y
void cnn_forward_scaled(Cnn& n, const double* s, float* out);
// an activation of the last forward pass as FP32 (test support)
gea_status cnn_copy_activation(Cnn& n, int which, float* out, gea_ptr_kind kind, std::string& err);

}  // namespace gea

// Kernels of the learned initial guess: a 3-D convolutional net on the
// coarse (N/2)^3 grid, channels-last activations [solve][point][16].
//
// Every layer is a periodic 3x3x3 convolution 16 -> 16 channels (inputs with
// fewer channels are zero-padded), BF16 weights and activations, FP32
// accumulation on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16) as an
// implicit GEMM: rows = 16 grid points, columns = 16 output channels, and the
// reduction runs over (neighbour, channel) pairs, two neighbours x 16
// channels per 32-wide MFMA step (27 neighbours padded to 28).
//
// The backward pass of a layer w.r.t. its input is the same convolution with
// spatially flipped, channel-transposed weights, so training reuses the
// forward kernel; weight gradients and Adam run on FP32 vector units.
#include "kernels.hpp"

namespace stern {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int C = kNetChannels;  // 16
constexpr int NB = 27;           // neighbours of a 3x3x3 stencil

__device__ __forceinline__ int nbr_index(int x, int y, int z, int n, int Nc) {
  const int dx = n / 9 - 1, dy = (n / 3) % 3 - 1, dz = n % 3 - 1;
  int a = x + dx, b = y + dy, c = z + dz;
  a += (a < 0) ? Nc : 0;
  a -= (a >= Nc) ? Nc : 0;
  b += (b < 0) ? Nc : 0;
  b -= (b >= Nc) ? Nc : 0;
  c += (c < 0) ? Nc : 0;
  c -= (c >= Nc) ? Nc : 0;
  return (a * Nc + b) * Nc + c;
}

// out[s][p][co] = act(bias[co] + sum_{n, ci} W[co][n][ci] in[s][nbr(p, n)][ci]); ACT: 0 none, 1 ReLU;
// OUT_F32: FP32 output (last layer, gradients), else BF16. Activations are
// stored with a per-solve stride of ldp >= npts points.
// Tiled form of the same convolution: a workgroup computes a 4 x 4 x 16 block
// of output points (16 rows of 16 consecutive z) of one solve. The periodic
// 6 x 6 x 18 halo of the input is staged once in LDS; wave w computes the
// rows of x = x0 + w. The MFMA takes the weights as its A operand and the
// activations as B, so D[cout][point] leaves 4 consecutive output channels of
// one point in each lane (one 8- or 16-byte store). Points past Nc in a
// partial tile are computed from wrapped inputs and not stored.
constexpr int kTX = 4, kTY = 4, kTZ = 16;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;

template <int ACT, bool OUT_F32>
__global__ __launch_bounds__(256) void k_conv3t(const __bf16* __restrict__ in, const __bf16* __restrict__ W,
                                                const float* __restrict__ bias, void* __restrict__ out, int Nc,
                                                int ldp) {
  __shared__ bf16x8 halo[kHX * kHY * kHZ][2];  // [point][channel half]
  const int s = blockIdx.y;
  const int nty = (Nc + kTY - 1) / kTY, ntz = (Nc + kTZ - 1) / kTZ;
  const int tile = blockIdx.x;
  const int tx = tile / (nty * ntz), ty = (tile / ntz) % nty, tz = tile % ntz;
  const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
  const __bf16* ins = in + (size_t)s * ldp * C;
  for (int i = threadIdx.x; i < kHX * kHY * kHZ * 2; i += 256) {
    const int h = i & 1, pt = i >> 1;
    const int px = pt / (kHY * kHZ), py = (pt / kHZ) % kHY, pz = pt % kHZ;
    int gx = x0 - 1 + px, gy = y0 - 1 + py, gz = z0 - 1 + pz;
    gx = ((gx % Nc) + Nc) % Nc;
    gy = ((gy % Nc) + Nc) % Nc;
    gz = ((gz % Nc) + Nc) % Nc;
    halo[pt][h] = *reinterpret_cast<const bf16x8*>(ins + (size_t)((gx * Nc + gy) * Nc + gz) * C + 8 * h);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, g = lane >> 4, half = g & 1;
  bf16x8 wf[14];
#pragma unroll
  for (int step = 0; step < 14; ++step) {
    const int n = 2 * step + (g >> 1);
    wf[step] = bf16x8{};
    if (n < NB) wf[step] = *reinterpret_cast<const bf16x8*>(W + ((size_t)l16 * NB + n) * C + 8 * half);
  }
  float bj[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bj[r] = bias ? bias[4 * g + r] : 0.f;
  __syncthreads();
  const int xl = wave;
  const int gxo = x0 + xl;
  for (int yl = 0; yl < kTY; ++yl) {
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int step = 0; step < 14; ++step) {
      const int n = 2 * step + (g >> 1);
      bf16x8 a = bf16x8{};
      if (n < NB) {
        const int dx = n / 9 - 1, dy = (n / 3) % 3 - 1, dz = n % 3 - 1;
        a = halo[((xl + 1 + dx) * kHY + (yl + 1 + dy)) * kHZ + (l16 + 1 + dz)][half];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[step], a, acc, 0, 0, 0);
    }
    // D[i][j]: column j = lane % 16 (point z0 + j), row i = 4 (lane / 16) + r (output channel)
    const int gyo = y0 + yl, gzo = z0 + l16;
    if (gxo < Nc && gyo < Nc && gzo < Nc) {
      const size_t o = ((size_t)s * ldp + (size_t)(gxo * Nc + gyo) * Nc + gzo) * C + 4 * g;
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[r] = acc[r] + bj[r];
        if (ACT == 1) v[r] = v[r] > 0.f ? v[r] : 0.f;
      }
      if (OUT_F32) {
        *reinterpret_cast<float4*>(reinterpret_cast<float*>(out) + o) = make_float4(v[0], v[1], v[2], v[3]);
      } else {
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        bf16x4 b;
#pragma unroll
        for (int r = 0; r < 4; ++r) b[r] = (__bf16)v[r];
        *reinterpret_cast<bf16x4*>(reinterpret_cast<__bf16*>(out) + o) = b;
      }
    }
  }
}

// dW[co][n][ci] = sum_{s, p} gout[s][p][co] in[s][nbr(p, n)][ci]; db[co] = sum gout.
// One workgroup per 4 x 4 x 16 tile of points, over all solves: the tile's
// input halo and output gradients are staged in LDS (FP32) and thread (co, ci)
// accumulates its 27 taps; the tile's partial goes to part[tile] and the tiles
// are summed in a fixed order afterwards.
__global__ __launch_bounds__(256) void k_conv3_wgrad(const __bf16* __restrict__ in, const float* __restrict__ gout,
                                                     float* __restrict__ part, int Nc, int ldp, int nsolve,
                                                     int ntiles) {
  __shared__ float hs[kHX * kHY * kHZ][C + 1];
  __shared__ float gs[kTX * kTY * kTZ][C + 1];
  const int nty = (Nc + kTY - 1) / kTY, ntz = (Nc + kTZ - 1) / kTZ;
  const int tile = blockIdx.x;
  const int tx = tile / (nty * ntz), ty = (tile / ntz) % nty, tz = tile % ntz;
  const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * kTZ;
  const int co = threadIdx.x >> 4, ci = threadIdx.x & 15;
  float acc[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) acc[n] = 0.f;
  float accb = 0.f;
  for (int s = 0; s < nsolve; ++s) {
    const __bf16* ins = in + (size_t)s * ldp * C;
    const float* gso = gout + (size_t)s * ldp * C;
    __syncthreads();  // the previous solve's reads of hs / gs are done
    for (int i = threadIdx.x; i < kHX * kHY * kHZ * C; i += 256) {
      const int c = i % C, pt = i / C;
      const int px = pt / (kHY * kHZ), py = (pt / kHZ) % kHY, pz = pt % kHZ;
      int gx = x0 - 1 + px, gy = y0 - 1 + py, gz = z0 - 1 + pz;
      gx = ((gx % Nc) + Nc) % Nc;
      gy = ((gy % Nc) + Nc) % Nc;
      gz = ((gz % Nc) + Nc) % Nc;
      hs[pt][c] = (float)ins[(size_t)((gx * Nc + gy) * Nc + gz) * C + c];
    }
    for (int i = threadIdx.x; i < kTX * kTY * kTZ * C; i += 256) {
      const int c = i % C, pt = i / C;
      const int lx = pt / (kTY * kTZ), ly = (pt / kTZ) % kTY, lz = pt % kTZ;
      const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
      float v = 0.f;  // points past Nc contribute nothing
      if (gx < Nc && gy < Nc && gz < Nc) v = gso[(size_t)((gx * Nc + gy) * Nc + gz) * C + c];
      gs[pt][c] = v;
    }
    __syncthreads();
    for (int pt = 0; pt < kTX * kTY * kTZ; ++pt) {
      const int lx = pt / (kTY * kTZ), ly = (pt / kTZ) % kTY, lz = pt % kTZ;
      const float gv = gs[pt][co];
      accb += gv;
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        const int dx = n / 9, dy = (n / 3) % 3, dz = n % 3;  // halo offsets 0..2 = d + 1
        acc[n] += gv * hs[((lx + dx) * kHY + (ly + dy)) * kHZ + (lz + dz)][ci];
      }
    }
  }
  // part layout: [ntiles][co][n][ci], then [ntiles][co] biases after the weights
#pragma unroll
  for (int n = 0; n < NB; ++n) part[(((size_t)tile * C + co) * NB + n) * C + ci] = acc[n];
  if (ci == 0) part[(size_t)ntiles * C * NB * C + (size_t)tile * C + co] = accb;
}

// sum the slices in order; grad = sum
__global__ void k_sum_slices(const float* __restrict__ part, int nslice, int nelem, float* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nelem) return;
  const int nw = C * NB * C;
  float a = 0.f;
  if (i < nw) {
    for (int s = 0; s < nslice; ++s) a += part[(size_t)s * nw + i];
  } else {
    const int co = i - nw;
    for (int s = 0; s < nslice; ++s) a += part[(size_t)nslice * nw + (size_t)s * C + co];
  }
  grad[i] = a;
}

// gin *= (act > 0)  (ReLU backward; act is the layer's BF16 output)
__global__ void k_relu_bwd(float* __restrict__ g, const __bf16* __restrict__ act, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!((float)act[i] > 0.f)) g[i] = 0.f;
}

__global__ void k_f32_to_bf16(const float* __restrict__ a, __bf16* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (__bf16)a[i];
}

// weights for the input gradient: Wt[ci][n'][co] = W[co][26 - n][ci]
__global__ void k_flip_weights(const float* __restrict__ W, __bf16* __restrict__ Wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C * NB * C) return;
  const int co = i / (NB * C), n = (i / C) % NB, ci = i % C;
  Wt[((size_t)ci * NB + (NB - 1 - n)) * C + co] = (__bf16)W[i];
}

// relative L2 loss per solve over channels 0,1: L_s = sum |out - t|^2 / sum |t|^2;
// gout = dL/dout (channels 0,1; other channels 0). loss_out[s] = L_s.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ out, const float* __restrict__ tgt,
                                              float* __restrict__ gout, float* __restrict__ loss_out, int npts,
                                              int ldp) {
  __shared__ float sh[2][4];
  const int s = blockIdx.x;
  const float* o = out + (size_t)s * ldp * C;
  const float* t = tgt + (size_t)s * ldp * 2;
  float num = 0.f, den = 0.f;
  for (int p = threadIdx.x; p < npts; p += 256) {
    const float d0 = o[(size_t)p * C] - t[2 * p], d1 = o[(size_t)p * C + 1] - t[2 * p + 1];
    num += d0 * d0 + d1 * d1;
    den += t[2 * p] * t[2 * p] + t[2 * p + 1] * t[2 * p + 1];
  }
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_xor(num, off);
    den += __shfl_xor(den, off);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = num;
    sh[1][threadIdx.x >> 6] = den;
  }
  __syncthreads();
  const float N0 = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
  const float D0 = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  const float inv = D0 > 0.f ? 1.f / D0 : 0.f;
  float* go = gout + (size_t)s * ldp * C;
  for (int p = threadIdx.x; p < ldp; p += 256) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      float v = 0.f;
      if (c < 2 && p < npts) v = 2.f * (o[(size_t)p * C + c] - t[2 * p + c]) * inv;
      go[(size_t)p * C + c] = v;
    }
  }
  if (threadIdx.x == 0) loss_out[s] = N0 * inv;
}

// Adam step (bias-corrected), gradients averaged over `scale` solves
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1, float c2,
                       float scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i] * scale;
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Net input of solve s: channels (Re psi, Im psi, Re b / |b|, Im b / |b|, eps_v, 0 ...)
// from coarse-grid fields psi_c [band][P] and b_c [s][P] (complex double).
__global__ void k_pack_input(const Z64* __restrict__ psi_c, const Z64* __restrict__ b_c,
                             const int* __restrict__ band, const double* __restrict__ eps,
                             const double* __restrict__ bnorm2, __bf16* __restrict__ out, int npts, int ldp) {
  const int s = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const Z64 ps = psi_c[(size_t)band[s] * npts + p];
  const Z64 bs = b_c[(size_t)s * npts + p];
  const double bn = bnorm2[s] > 0.0 ? 1.0 / sqrt(bnorm2[s]) : 0.0;
  __bf16* o = out + ((size_t)s * ldp + p) * C;
  float v[C];
#pragma unroll
  for (int c = 0; c < C; ++c) v[c] = 0.f;
  v[0] = (float)ps.re;
  v[1] = (float)ps.im;
  v[2] = (float)(bs.re * bn);
  v[3] = (float)(bs.im * bn);
  v[4] = (float)eps[s];
#pragma unroll
  for (int c = 0; c < C; ++c) o[c] = (__bf16)v[c];
}

// Band input of the preconditioner features: channels (Re psi_v, Im psi_v, 0, 0, eps_v, 0 ...)
__global__ void k_pack_band(const Z64* __restrict__ psi_c, const double* __restrict__ eps,
                            __bf16* __restrict__ out, int npts, int ldp) {
  const int v = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const Z64 ps = psi_c[(size_t)v * npts + p];
  __bf16* o = out + ((size_t)v * ldp + p) * C;
  float w[C];
#pragma unroll
  for (int c = 0; c < C; ++c) w[c] = 0.f;
  w[0] = (float)ps.re;
  w[1] = (float)ps.im;
  w[4] = (float)eps[v];
#pragma unroll
  for (int c = 0; c < C; ++c) o[c] = (__bf16)w[c];
}

// training target of solve s: x~(r) / |b| on the coarse grid, [s][P][2] float
__global__ void k_pack_target(const Z64* __restrict__ x_c, const double* __restrict__ bnorm2,
                              float* __restrict__ tgt, int npts, int ldp) {
  const int s = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const double bn = bnorm2[s] > 0.0 ? 1.0 / sqrt(bnorm2[s]) : 0.0;
  const Z64 v = x_c[(size_t)s * npts + p];
  tgt[((size_t)s * ldp + p) * 2] = (float)(v.re * bn);
  tgt[((size_t)s * ldp + p) * 2 + 1] = (float)(v.im * bn);
}

// net output (channels 0,1, FP32) -> complex coarse field x~(r) |b|
__global__ void k_unpack_output(const float* __restrict__ out, const double* __restrict__ bnorm2,
                                Z64* __restrict__ x_c, int npts, int ldp) {
  const int s = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const double bn = sqrt(bnorm2[s]);
  const float* o = out + ((size_t)s * ldp + p) * C;
  x_c[(size_t)s * npts + p] = zmk((double)o[0] * bn, (double)o[1] * bn);
}

// ---- learned diagonal preconditioner head ----
// K_s(G) = Teter(y) * softplus(z_s(u)) / ln 2 with y = |G|^2 / (2 T_v), u = log2 y
// clamped to the knot range, and z_s the piecewise-linear interpolation of the
// solve's kPrecKnots coefficients c_s on knots u_k = kPrecU0 + k kPrecDu. At c = 0
// the scale is exactly 1 (Teter). c_s = bh + Wh f_s, f_s = (mean over grid points
// of the second hidden layer's 16 channels, eps_v, T_v).

// Teter-Payne-Allan kinetic preconditioner (Phys. Rev. B 40, 12255 (1989))
__device__ __forceinline__ double teter_k(double y) {
  const double n = 27.0 + y * (18.0 + y * (12.0 + 8.0 * y));
  return n / (n + 16.0 * y * y * y * y);
}

struct KnotPos {
  int k0;
  double w;
};
__device__ __forceinline__ KnotPos knot_pos(double y) {
  double u = log2(fmax(y, 1e-300));
  const double umax = kPrecU0 + kPrecDu * (kPrecKnots - 1);
  u = fmin(fmax(u, (double)kPrecU0), umax);
  double t = (u - kPrecU0) / kPrecDu;
  int k0 = (int)floor(t);
  if (k0 > kPrecKnots - 2) k0 = kPrecKnots - 2;
  return KnotPos{k0, t - k0};
}

__device__ __forceinline__ double softplus(double z) { return z > 30.0 ? z : log1p(exp(z)); }

// f[s][0..15] = mean of act[s][p][c] over the npts grid points; f[s][16] = eps, f[s][17] = 1 / invT
__global__ __launch_bounds__(256) void k_pool(const __bf16* __restrict__ act, const double* __restrict__ eps,
                                              const double* __restrict__ invT, float* __restrict__ f, int npts,
                                              int ldp) {
  __shared__ float sh[16][17];
  const int s = blockIdx.x;
  const int c = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const __bf16* a = act + (size_t)s * ldp * C;
  float acc = 0.f;
  for (int p = grp; p < npts; p += 16) acc += (float)a[(size_t)p * C + c];
  sh[grp][c] = acc;
  __syncthreads();
  if (threadIdx.x < 16) {
    float t = 0.f;
    for (int g = 0; g < 16; ++g) t += sh[g][threadIdx.x];
    f[(size_t)s * kPrecIn + threadIdx.x] = t / (float)npts;
  } else if (threadIdx.x == 16) {
    f[(size_t)s * kPrecIn + 16] = (float)eps[s];
  } else if (threadIdx.x == 17) {
    f[(size_t)s * kPrecIn + 17] = (float)(1.0 / invT[s]);
  }
}

// coef[s][k] = bh[k] + sum_j Wh[k][j] f[s][j]   (head = Wh [kPrecKnots][kPrecIn], bh [kPrecKnots])
__global__ void k_prec_coef(const float* __restrict__ head, const float* __restrict__ f, float* __restrict__ coef,
                            int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * kPrecKnots) return;
  const int s = i / kPrecKnots, k = i % kPrecKnots;
  float a = head[kPrecKnots * kPrecIn + k];
  for (int j = 0; j < kPrecIn; ++j) a += head[k * kPrecIn + j] * f[(size_t)s * kPrecIn + j];
  coef[i] = a;
}

// K[s][G] for G < npw_pad (T_v from the features)
__global__ void k_prec_build(const float* __restrict__ coef, const float* __restrict__ f,
                             const double* __restrict__ g2h, float* __restrict__ K, int npw_pad) {
  const int s = blockIdx.y;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw_pad) return;
  const double y = g2h[g] / (double)f[(size_t)s * kPrecIn + 17];
  const KnotPos kp = knot_pos(y);
  const double z = (double)coef[s * kPrecKnots + kp.k0] * (1.0 - kp.w) + (double)coef[s * kPrecKnots + kp.k0 + 1] * kp.w;
  K[(size_t)s * npw_pad + g] = (float)(teter_k(y) * softplus(z) * 1.4426950408889634);  // / ln 2
}

// out[t] = K[t] o R0[idx[t]]
__global__ void k_prec_apply(const float* __restrict__ K, const Z64* __restrict__ R0, const int* __restrict__ idx,
                             Z64* __restrict__ out, int npw_pad) {
  const int t = blockIdx.y;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw_pad) return;
  const Z64 r = R0[(size_t)idx[t] * npw_pad + g];
  const double k = (double)K[(size_t)t * npw_pad + g];
  out[(size_t)t * npw_pad + g] = zmk(k * r.re, k * r.im);
}

__device__ __forceinline__ double block_sum256(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

// Loss L_t = ||P_t - e0||^2 / ||e0||^2 with P_t = P_c (K o r0) (given), and
// gc[t][k] = dL_t / dc_{t,k}. P_c is self-adjoint and e0 lies in its range, so
// dL/dK(G) = 2 Re(conj r0(G) (P - e0)(G)) / ||e0||^2.
__global__ __launch_bounds__(256) void k_prec_grad(const Z64* __restrict__ P, const Z64* __restrict__ R0,
                                                   const Z64* __restrict__ E0, const int* __restrict__ idx,
                                                   const float* __restrict__ coef, const float* __restrict__ f,
                                                   const double* __restrict__ g2h, int npw, int npw_pad,
                                                   float* __restrict__ gc, float* __restrict__ loss) {
  __shared__ double sh[4];
  const int t = blockIdx.x;
  const size_t oj = (size_t)idx[t] * npw_pad, ot = (size_t)t * npw_pad;
  const double T = (double)f[(size_t)t * kPrecIn + 17];
  double ee = 0.0, dd = 0.0;
  for (int g = threadIdx.x; g < npw; g += 256) {
    const Z64 e = E0[oj + g], p = P[ot + g];
    ee += e.re * e.re + e.im * e.im;
    dd += (p.re - e.re) * (p.re - e.re) + (p.im - e.im) * (p.im - e.im);
  }
  ee = block_sum256(ee, sh);
  dd = block_sum256(dd, sh);
  const double inv = ee > 0.0 ? 1.0 / ee : 0.0;
  double acc[kPrecKnots];
#pragma unroll
  for (int k = 0; k < kPrecKnots; ++k) acc[k] = 0.0;
  for (int g = threadIdx.x; g < npw; g += 256) {
    const Z64 e = E0[oj + g], p = P[ot + g], r = R0[oj + g];
    const double y = g2h[g] / T;
    const KnotPos kp = knot_pos(y);
    const double z = (double)coef[t * kPrecKnots + kp.k0] * (1.0 - kp.w) + (double)coef[t * kPrecKnots + kp.k0 + 1] * kp.w;
    const double sig = 1.0 / (1.0 + exp(-z));
    const double dK = 2.0 * (r.re * (p.re - e.re) + r.im * (p.im - e.im)) * inv;
    const double dz = dK * teter_k(y) * sig * 1.4426950408889634;
#pragma unroll
    for (int k = 0; k < kPrecKnots; ++k) {
      if (k == kp.k0) acc[k] += dz * (1.0 - kp.w);
      if (k == kp.k0 + 1) acc[k] += dz * kp.w;
    }
  }
#pragma unroll
  for (int k = 0; k < kPrecKnots; ++k) {
    const double v = block_sum256(acc[k], sh);
    if (threadIdx.x == 0) gc[t * kPrecKnots + k] = (float)v;
  }
  if (threadIdx.x == 0) loss[t] = (float)(dd * inv);
}

// head gradient: dWh[k][j] = sum_t gc[t][k] f[t][j]; dbh[k] = sum_t gc[t][k]
__global__ void k_head_grad(const float* __restrict__ gc, const float* __restrict__ f, int n,
                            float* __restrict__ grad) {
  const int i = threadIdx.x;
  if (i >= kPrecParams) return;
  float a = 0.f;
  if (i < kPrecKnots * kPrecIn) {
    const int k = i / kPrecIn, j = i % kPrecIn;
    for (int t = 0; t < n; ++t) a += gc[t * kPrecKnots + k] * f[(size_t)t * kPrecIn + j];
  } else {
    const int k = i - kPrecKnots * kPrecIn;
    for (int t = 0; t < n; ++t) a += gc[t * kPrecKnots + k];
  }
  grad[i] = a;
}

// dst[j] = src[rows[j]] (sub = 0) or src[rows[j]] - dst[j] (sub = 1), rows of ld complex values
__global__ void k_gather_rows(Z64* __restrict__ dst, const Z64* __restrict__ src, const int* __restrict__ rows,
                              int ld, int sub) {
  const int j = blockIdx.y;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ld) return;
  const Z64 v = src[(size_t)rows[j] * ld + g];
  Z64* d = dst + (size_t)j * ld + g;
  *d = sub ? zmk(v.re - d->re, v.im - d->im) : v;
}

__global__ void k_gather_f32(float* __restrict__ dst, const float* __restrict__ src, const int* __restrict__ rows,
                             int ld, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * ld) return;
  dst[i] = src[(size_t)rows[i / ld] * ld + i % ld];
}

}  // namespace

int net_ldp(int Nc) { return (Nc * Nc * Nc + 15) / 16 * 16; }

void launch_conv3(const __bf16* in, const __bf16* W, const float* bias, void* out, int Nc, int nsolve, int act,
                  bool out_f32, hipStream_t st) {
  if (nsolve <= 0) return;
  const int ldp = net_ldp(Nc);
  const int ntiles = ((Nc + kTX - 1) / kTX) * ((Nc + kTY - 1) / kTY) * ((Nc + kTZ - 1) / kTZ);
  const dim3 grid(ntiles, nsolve);
  if (act == 1 && !out_f32)
    k_conv3t<1, false><<<grid, 256, 0, st>>>(in, W, bias, out, Nc, ldp);
  else if (act == 0 && out_f32)
    k_conv3t<0, true><<<grid, 256, 0, st>>>(in, W, bias, out, Nc, ldp);
  else if (act == 0 && !out_f32)
    k_conv3t<0, false><<<grid, 256, 0, st>>>(in, W, bias, out, Nc, ldp);
  else
    k_conv3t<1, true><<<grid, 256, 0, st>>>(in, W, bias, out, Nc, ldp);
}

int conv3_wgrad_parts(int Nc) {
  return ((Nc + kTX - 1) / kTX) * ((Nc + kTY - 1) / kTY) * ((Nc + kTZ - 1) / kTZ);
}

void launch_conv3_wgrad(const __bf16* in, const float* gout, float* part, float* grad, int Nc, int nsolve,
                        hipStream_t st) {
  const int ntiles = conv3_wgrad_parts(Nc);
  k_conv3_wgrad<<<ntiles, 256, 0, st>>>(in, gout, part, Nc, net_ldp(Nc), nsolve, ntiles);
  const int nelem = C * NB * C + C;
  k_sum_slices<<<(nelem + 255) / 256, 256, 0, st>>>(part, ntiles, nelem, grad);
}

void launch_relu_bwd(float* g, const __bf16* act, size_t n, hipStream_t st) {
  k_relu_bwd<<<(unsigned)std::min<size_t>((n + 255) / 256, 65536), 256, 0, st>>>(g, act, n);
}
void launch_f32_to_bf16(const float* a, __bf16* b, size_t n, hipStream_t st) {
  k_f32_to_bf16<<<(unsigned)std::min<size_t>((n + 255) / 256, 65536), 256, 0, st>>>(a, b, n);
}
void launch_flip_weights(const float* W, __bf16* Wt, hipStream_t st) {
  k_flip_weights<<<(C * NB * C + 255) / 256, 256, 0, st>>>(W, Wt);
}
void launch_loss(const float* out, const float* tgt, float* gout, float* loss, int Nc, int nsolve, hipStream_t st) {
  if (nsolve > 0) k_loss<<<nsolve, 256, 0, st>>>(out, tgt, gout, loss, Nc * Nc * Nc, net_ldp(Nc));
}
void launch_adam(float* w, float* m, float* v, const float* g, int n, float lr, int step, float scale,
                 hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  k_adam<<<(n + 255) / 256, 256, 0, st>>>(w, m, v, g, n, lr, b1, b2, 1e-8f, c1, c2, scale);
}
void launch_pack_input(const Z64* psi_c, const Z64* b_c, const int* band, const double* eps, const double* bnorm2,
                       __bf16* out, int Nc, int nsolve, hipStream_t st) {
  const int npts = Nc * Nc * Nc;
  if (nsolve > 0)
    k_pack_input<<<dim3((npts + 255) / 256, nsolve), 256, 0, st>>>(psi_c, b_c, band, eps, bnorm2, out, npts,
                                                                   net_ldp(Nc));
}
void launch_pack_band(const Z64* psi_c, const double* eps, __bf16* out, int Nc, int nband, hipStream_t st) {
  const int npts = Nc * Nc * Nc;
  if (nband > 0) k_pack_band<<<dim3((npts + 255) / 256, nband), 256, 0, st>>>(psi_c, eps, out, npts, net_ldp(Nc));
}
void launch_pack_target(const Z64* x_c, const double* bnorm2, float* tgt, int Nc, int nsolve, hipStream_t st) {
  const int npts = Nc * Nc * Nc;
  if (nsolve > 0)
    k_pack_target<<<dim3((npts + 255) / 256, nsolve), 256, 0, st>>>(x_c, bnorm2, tgt, npts, net_ldp(Nc));
}
void launch_unpack_output(const float* out, const double* bnorm2, Z64* x_c, int Nc, int nsolve, hipStream_t st) {
  const int npts = Nc * Nc * Nc;
  if (nsolve > 0)
    k_unpack_output<<<dim3((npts + 255) / 256, nsolve), 256, 0, st>>>(out, bnorm2, x_c, npts, net_ldp(Nc));
}

void launch_pool(const __bf16* act, const double* eps, const double* invT, float* f, int Nc, int nsolve,
                 hipStream_t st) {
  if (nsolve > 0) k_pool<<<nsolve, 256, 0, st>>>(act, eps, invT, f, Nc * Nc * Nc, net_ldp(Nc));
}
void launch_prec_coef(const float* head, const float* f, float* coef, int n, hipStream_t st) {
  if (n > 0) k_prec_coef<<<(n * kPrecKnots + 255) / 256, 256, 0, st>>>(head, f, coef, n);
}
void launch_prec_build(const float* coef, const float* f, const double* g2h, float* K, int npw_pad, int n,
                       hipStream_t st) {
  if (n > 0) k_prec_build<<<dim3((npw_pad + 255) / 256, n), 256, 0, st>>>(coef, f, g2h, K, npw_pad);
}
void launch_prec_apply(const float* K, const Z64* R0, const int* idx, Z64* out, int npw_pad, int n, hipStream_t st) {
  if (n > 0) k_prec_apply<<<dim3((npw_pad + 255) / 256, n), 256, 0, st>>>(K, R0, idx, out, npw_pad);
}
void launch_prec_grad(const Z64* P, const Z64* R0, const Z64* E0, const int* idx, const float* coef, const float* f,
                      const double* g2h, int npw, int npw_pad, float* gc, float* loss, int n, hipStream_t st) {
  if (n > 0) k_prec_grad<<<n, 256, 0, st>>>(P, R0, E0, idx, coef, f, g2h, npw, npw_pad, gc, loss);
}
void launch_head_grad(const float* gc, const float* f, int n, float* grad, hipStream_t st) {
  k_head_grad<<<1, 256, 0, st>>>(gc, f, n, grad);
}
void launch_gather_rows(Z64* dst, const Z64* src, const int* rows, int ld, int n, bool sub, hipStream_t st) {
  if (n > 0) k_gather_rows<<<dim3((ld + 255) / 256, n), 256, 0, st>>>(dst, src, rows, ld, sub ? 1 : 0);
}
void launch_gather_f32(float* dst, const float* src, const int* rows, int ld, int n, hipStream_t st) {
  if (n > 0) k_gather_f32<<<(n * ld + 255) / 256, 256, 0, st>>>(dst, src, rows, ld, n);
}

}  // namespace stern

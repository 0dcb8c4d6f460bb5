// k_backward.hip -- gradients of an image loss with respect to per-vertex
// colours and texels for Gouraud and textured shading.  For each covered
// pixel with upstream gradient G (alpha ignored) and saved perspective
// barycentrics (b0, b1, b2):
//   untextured: dC[v_k][c] += b_k G_c
//   textured:   dC[v_k][c] += b_k G_c T_c ,  dTex[j][c] += w_j G_c Cint_c
// Coverage is not differentiated.  Scatters are float32 global atomics.
#include "pk_internal.h"

#pragma clang fp contract(off)

namespace pk {

__global__ __launch_bounds__(256) void k_backward(Geom G, Shade sh, const int32_t *primid,
                                                  const float *bary, const float *grad,
                                                  float *gv, float *gt) {
    const int64_t npix = (int64_t)G.S * G.W * G.H;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const int32_t t = primid[p];
    if (t < 0) return;
    const int32_t s = (int32_t)(p / ((int64_t)G.W * G.H));
    int64_t g, vb;
    if (G.S == 1 || G.instanced) { g = t; vb = 0; }
    else { g = (int64_t)G.tri_off[s] + t; vb = G.vtx_off[s]; }
    int64_t v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = vb + (G.idx ? (int64_t)G.idx[3 * g + k] : 3 * (int64_t)t + k);
    const float2 bb = reinterpret_cast<const float2 *>(bary)[p];
    const float b1 = bb.x, b2 = bb.y, b0 = (1.0f - b1) - b2;
    const float4 Gc = reinterpret_cast<const float4 *>(grad)[p];
    const float gc[3] = {Gc.x, Gc.y, Gc.z};
    const int64_t V = G.V;
    if (sh.shading == PK_SHADE_TEXTURED) {
        float rgb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float *pl = sh.color + c * V;
            float acc = b0 * pl[v[0]];
            acc = acc + b1 * pl[v[1]];
            acc = acc + b2 * pl[v[2]];
            rgb[c] = acc;
        }
        float u = b0 * sh.uv[v[0]];
        u = u + b1 * sh.uv[v[1]];
        u = u + b2 * sh.uv[v[2]];
        float vv = b0 * sh.uv[V + v[0]];
        vv = vv + b1 * sh.uv[V + v[1]];
        vv = vv + b2 * sh.uv[V + v[2]];
        const float su = u * (float)sh.tex_w - 0.5f, sv = vv * (float)sh.tex_h - 0.5f;
        const float fi = floorf(su), fj = floorf(sv);
        const float fs = su - fi, ft = sv - fj;
        const float ci = fminf(fmaxf(fi, -1.0f), (float)sh.tex_w);
        const float cj = fminf(fmaxf(fj, -1.0f), (float)sh.tex_h);
        const int i0 = min(max((int)ci, 0), sh.tex_w - 1), i1 = min(max((int)ci + 1, 0), sh.tex_w - 1);
        const int j0 = min(max((int)cj, 0), sh.tex_h - 1), j1 = min(max((int)cj + 1, 0), sh.tex_h - 1);
        const float w[4] = {(1.0f - fs) * (1.0f - ft), fs * (1.0f - ft), (1.0f - fs) * ft, fs * ft};
        const int64_t tx[4] = {(int64_t)j0 * sh.tex_w + i0, (int64_t)j0 * sh.tex_w + i1,
                               (int64_t)j1 * sh.tex_w + i0, (int64_t)j1 * sh.tex_w + i1};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float T = w[0] * sh.texture[3 * tx[0] + c];
            T = T + w[1] * sh.texture[3 * tx[1] + c];
            T = T + w[2] * sh.texture[3 * tx[2] + c];
            T = T + w[3] * sh.texture[3 * tx[3] + c];
            const float gT = gc[c] * T;
            atomicAdd(gv + c * V + v[0], b0 * gT);
            atomicAdd(gv + c * V + v[1], b1 * gT);
            atomicAdd(gv + c * V + v[2], b2 * gT);
            const float gC = gc[c] * rgb[c];
#pragma unroll
            for (int j = 0; j < 4; ++j) atomicAdd(gt + 3 * tx[j] + c, w[j] * gC);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            atomicAdd(gv + c * V + v[0], b0 * gc[c]);
            atomicAdd(gv + c * V + v[1], b1 * gc[c]);
            atomicAdd(gv + c * V + v[2], b2 * gc[c]);
        }
    }
}

hipError_t launch_backward(const Geom &G, const Shade &sh, const int32_t *primid,
                           const float *bary, const float *grad, float *grad_vcolor,
                           float *grad_tex, hipStream_t st) {
    const int64_t npix = (int64_t)G.S * G.W * G.H;
    if (npix == 0) return hipSuccess;
    hipLaunchKernelGGL(k_backward, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, G, sh,
                       primid, bary, grad, grad_vcolor, grad_tex);
    return hipGetLastError();
}

}  // namespace pk

// Per-bin precomputation before the iterations (Algorithm 2, before the loop).
//
// For every bin, from the complex64 observation x_ij and the FP64 row
// constants of the setup kernel, in FP64:
//   z       = G x           (G = F^H, F F^H = (R')^+)
//   tau^ax  = g^H z         = a^H (R')^+ x                      eq. (47)
//   sigma^bx= b^H x                                              eq. (33)
//   tau^xx  = |z|^2         = x^H (R')^+ x                      eq. (48)
//   nu      = |z - (tau^ax / tau^aa) g|^2 = tau^xx - |tau^ax|^2 / tau^aa
// nu is the part of tau^xx orthogonal to a in the (R')^+ metric, kept as a
// sum of squares so the float iteration never subtracts large terms.
// Stored as float4 {tau^ax, sigma^bx} and float nu (20 bytes per bin).
//
// Memory-bound: reads 8M bytes and writes 20 bytes per bin; one bin per
// lane, consecutive lanes on consecutive frames (coalesced), row constants
// staged in LDS.  One launch per microphone count M.
#include "rcscm_internal.h"

namespace rcscm {

namespace {

template <int M>
__global__ __launch_bounds__(256) void precompute_kernel(const ChunkInfo* __restrict__ chunks,
                                                         const RowInfo* __restrict__ rows,
                                                         const RowConstD* __restrict__ rcd,
                                                         const float2* __restrict__ x,
                                                         float4* __restrict__ tsig,
                                                         float* __restrict__ nu,
                                                         unsigned* __restrict__ status) {
  const ChunkInfo ck = chunks[blockIdx.x];
  const RowInfo ri = rows[ck.row];
  const RowConstD* D = rcd + ck.row;

  __shared__ double2 sG[M * M];
  __shared__ double2 sg[M], sb[M];
  __shared__ double s_taa;
  const int t = threadIdx.x;
  if (t < M * M) sG[t] = D->G[(t / M) * MAXM + (t % M)];
  if (t < M) {
    sg[t] = D->g[t];
    sb[t] = D->b[t];
  }
  if (t == 0) s_taa = D->t_aa;
  __syncthreads();
  const double taa = s_taa;
  const double inv_taa = taa > 0.0 ? 1.0 / taa : 0.0;

  bool bad = false;
  for (int jj = t; jj < ck.len; jj += blockDim.x) {
    const int j = ck.start + jj;
    const float2* xp = x + ri.x_off + (long long)j * M;
    double xr[M], xi[M];
    if ((M & 1) == 0 && (ri.x_off & 1) == 0) {  // 16-byte aligned pairs of mics
      const float4* xp4 = reinterpret_cast<const float4*>(xp);
#pragma unroll
      for (int m = 0; m < M / 2; ++m) {
        const float4 v = xp4[m];
        xr[2 * m] = v.x;
        xi[2 * m] = v.y;
        xr[2 * m + 1] = v.z;
        xi[2 * m + 1] = v.w;
      }
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const float2 v = xp[m];
        xr[m] = v.x;
        xi[m] = v.y;
      }
    }
    // keep G in LDS (re-read per bin) instead of M*M*4 registers
    asm volatile("" ::: "memory");
    double zr[M], zi[M];
#pragma unroll
    for (int p = 0; p < M; ++p) {
      double ar = 0.0, ai = 0.0;
#pragma unroll
      for (int n = 0; n < M; ++n) {
        const double2 gpn = sG[p * M + n];
        ar = fma(gpn.x, xr[n], fma(-gpn.y, xi[n], ar));
        ai = fma(gpn.x, xi[n], fma(gpn.y, xr[n], ai));
      }
      zr[p] = ar;
      zi[p] = ai;
    }
    double tax_r = 0.0, tax_i = 0.0, sbx_r = 0.0, sbx_i = 0.0, txx = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      // conj(g) z, conj(b) x
      tax_r = fma(sg[m].x, zr[m], fma(sg[m].y, zi[m], tax_r));
      tax_i = fma(sg[m].x, zi[m], fma(-sg[m].y, zr[m], tax_i));
      sbx_r = fma(sb[m].x, xr[m], fma(sb[m].y, xi[m], sbx_r));
      sbx_i = fma(sb[m].x, xi[m], fma(-sb[m].y, xr[m], sbx_i));
      txx = fma(zr[m], zr[m], fma(zi[m], zi[m], txx));
    }
    double nuv;
    if (taa > 0.0) {
      const double kr = tax_r * inv_taa, ki = tax_i * inv_taa;
      nuv = 0.0;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        // z - k g
        const double dr = zr[m] - (kr * sg[m].x - ki * sg[m].y);
        const double di = zi[m] - (kr * sg[m].y + ki * sg[m].x);
        nuv = fma(dr, dr, fma(di, di, nuv));
      }
    } else {
      nuv = txx;
    }
    const long long bin = ri.bin_off + j;
    tsig[bin] = make_float4((float)tax_r, (float)tax_i, (float)sbx_r, (float)sbx_i);
    nu[bin] = (float)nuv;
    bad = bad || !isfinite(txx) || !isfinite(sbx_r) || !isfinite(sbx_i);
  }
  if (bad) atomicOr(status + ck.row, ST_NONFINITE_IN);
}

template <int M>
void launch_m(hipStream_t s, int nchunks, const ChunkInfo* chunks, const RowInfo* rows,
              const RowConstD* rcd, const float2* x, float4* tsig, float* nu, unsigned* status) {
  hipLaunchKernelGGL(precompute_kernel<M>, dim3(nchunks), dim3(256), 0, s, chunks, rows, rcd, x,
                     tsig, nu, status);
}

}  // namespace

void launch_precompute(hipStream_t s, int M, int nchunks, const ChunkInfo* chunks,
                       const RowInfo* rows, const RowConstD* rcd, const float2* x, float4* tsig,
                       float* nu, unsigned* status) {
  if (nchunks <= 0) return;
  switch (M) {
    case 2: launch_m<2>(s, nchunks, chunks, rows, rcd, x, tsig, nu, status); break;
    case 3: launch_m<3>(s, nchunks, chunks, rows, rcd, x, tsig, nu, status); break;
    case 4: launch_m<4>(s, nchunks, chunks, rows, rcd, x, tsig, nu, status); break;
    case 5: launch_m<5>(s, nchunks, chunks, rows, rcd, x, tsig, nu, status); break;
    case 6: launch_m<6>(s, nchunks, chunks, rows, rcd, x, tsig, nu, status); break;
    case 7: launch_m<7>(s, nchunks, chunks, rows, rcd, x, tsig, nu, status); break;
    case 8: launch_m<8>(s, nchunks, chunks, rows, rcd, x, tsig, nu, status); break;
    default: break;
  }
}

}  // namespace rcscm

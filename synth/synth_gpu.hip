// Device build of the row generator in synth.c (same Philox4x32-10 streams,
// same alias table, same acceptance rule), so the 200M-row shard can be made
// in HBM directly.  Rows are bit-identical to the host generator's; only
// Poisson row sizes are supported here (the lognormal law uses libm on the
// host).  Input generation only: none of the similarity method is here.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define EXPORT extern "C" __attribute__((visibility("default")))

namespace {

__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                       uint32_t out[4]) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

struct Stream {
  uint32_t k0, k1, o0, o1, tag, blk;
  uint32_t buf[4];
  __device__ Stream(uint64_t key, uint64_t owner, uint32_t t)
      : k0((uint32_t)key), k1((uint32_t)(key >> 32)), o0((uint32_t)owner), o1((uint32_t)(owner >> 32)), tag(t),
        blk(0xFFFFFFFFu) {}
  __device__ uint64_t draw(uint32_t j) {
    uint32_t b = j >> 1;
    if (b != blk) {
      philox(o0, o1, tag, b, k0, k1, buf);
      blk = b;
    }
    return (j & 1) ? (((uint64_t)buf[3] << 32) | buf[2]) : (((uint64_t)buf[1] << 32) | buf[0]);
  }
};

__global__ void k_nnz(uint64_t key, uint64_t row0, uint64_t n, const double* pcdf, uint32_t pcdf_n, uint32_t lo,
                      uint32_t hi, uint32_t* out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    Stream s(key, row0 + i, 1u);
    double u = (double)(s.draw(0) >> 11) * 0x1.0p-53;
    uint32_t k = 0;
    while (k < pcdf_n && !(u < pcdf[k])) ++k;
    out[i] = k < lo ? lo : (k > hi ? hi : k);
  }
}

__global__ void k_fill(uint64_t key, uint64_t row0, uint64_t n, uint32_t dim, int zipf, const uint64_t* __restrict__ tab,
                       const int64_t* __restrict__ indptr, int32_t* __restrict__ indices) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const int64_t base = indptr[i] - indptr[0];
    const uint32_t nnz = (uint32_t)(indptr[i + 1] - indptr[i]);
    int32_t* out = indices + base;
    Stream s(key, row0 + i, 2u);
    uint32_t got = 0, j = 0;
    while (got < nnz) {
      uint64_t x = s.draw(j++);
      uint32_t col = (uint32_t)(((x >> 32) * (uint64_t)dim) >> 32);
      uint32_t v = col;
      if (zipf) {
        uint64_t e = tab[col];
        v = ((uint32_t)x < (uint32_t)e) ? col : (uint32_t)(e >> 32);
      }
      bool dup = false;
      for (uint32_t q = 0; q < got; ++q) dup |= (uint32_t)out[q] == v;
      if (!dup) out[got++] = (int32_t)v;
    }
  }
}

}  // namespace

EXPORT int synth_gpu_rows_nnz(uint64_t key, uint64_t row0, uint64_t n, const double* pcdf, uint32_t pcdf_n,
                              uint32_t lo, uint32_t hi, uint32_t* out, void* stream) {
  if (n == 0) return 0;
  uint64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_nnz, dim3((uint32_t)g), dim3(256), 0, (hipStream_t)stream, key, row0, n, pcdf, pcdf_n, lo, hi,
                     out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

EXPORT int synth_gpu_rows_fill(uint64_t key, uint64_t row0, uint64_t n, uint32_t dim, int zipf, const uint64_t* tab,
                               const int64_t* indptr, int32_t* indices, void* stream) {
  if (n == 0) return 0;
  uint64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fill, dim3((uint32_t)g), dim3(256), 0, (hipStream_t)stream, key, row0, n, dim, zipf, tab,
                     indptr, indices);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

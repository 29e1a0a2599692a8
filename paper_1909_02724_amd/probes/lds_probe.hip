// LDS read-bandwidth probe for the back-projection roofline. Every lane
// reads 16 B per ds_read_b128 from conflict-free contiguous addresses, two
// 64 KB workgroups per CU, 2048 workgroups; prints TB/s and bytes per clock
// per CU at 2.4 GHz. bench.py takes its LDS peak from this measurement.
// Build: hipcc -O3 --offload-arch=gfx950 lds_probe.hip -o lds_probe
#include <hip/hip_runtime.h>
#include <cstdio>
__global__ __launch_bounds__(256) void lds_bw(float4* out, int iters) {
  __shared__ float4 buf[4096];  // 64 KB
  for (int k = threadIdx.x; k < 4096; k += 256) buf[k] = make_float4(k, k + 1, k + 2, k + 3);
  __syncthreads();
  float4 a = make_float4(0, 0, 0, 0), b = a, c = a, d = a;
  const unsigned lane = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    const unsigned base = (unsigned)(it * 256);
    float4 x0 = buf[(lane + base) & 4095];
    float4 x1 = buf[(lane + base + 1024) & 4095];
    float4 x2 = buf[(lane + base + 2048) & 4095];
    float4 x3 = buf[(lane + base + 3072) & 4095];
    a.x += x0.x; a.y += x0.y; a.z += x0.z; a.w += x0.w;
    b.x += x1.x; b.y += x1.y; b.z += x1.z; b.w += x1.w;
    c.x += x2.x; c.y += x2.y; c.z += x2.z; c.w += x2.w;
    d.x += x3.x; d.y += x3.y; d.z += x3.z; d.w += x3.w;
  }
  out[blockIdx.x * 256 + threadIdx.x] = make_float4(a.x + b.x + c.x + d.x, a.y + b.y + c.y + d.y,
                                                    a.z + b.z + c.z + d.z, a.w + b.w + c.w + d.w);
}
int main() {
  const int blocks = 256 * 8, iters = 4096;
  float4* out;
  if (hipMalloc(&out, sizeof(float4) * blocks * 256) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  hipEventCreate(&e0); hipEventCreate(&e1);
  hipLaunchKernelGGL(lds_bw, dim3(blocks), dim3(256), 0, 0, out, 64);
  hipDeviceSynchronize();
  hipEventRecord(e0);
  hipLaunchKernelGGL(lds_bw, dim3(blocks), dim3(256), 0, 0, out, iters);
  hipEventRecord(e1);
  if (hipEventSynchronize(e1) != hipSuccess) return 2;
  float ms; hipEventElapsedTime(&ms, e0, e1);
  const double bytes = (double)blocks * 256 * iters * 4 * 16;
  printf("lds_bw: %.3f ms, %.1f TB/s, %.1f B/clk/CU at 2.4 GHz\n", ms, bytes / ms / 1e9, bytes / (ms * 1e-3) / 256 / 2.4e9);
  hipFree(out);
  return 0;
}

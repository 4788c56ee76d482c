// Plain device copy of a known size, used to scale the FETCH_SIZE and
// WRITE_SIZE counters (bytes read / written per dispatch) into HBM bytes.
//
//   hipcc --offload-arch=gfx950 -O3 copy_probe.hip -o copy_probe && ./copy_probe
#include <hip/hip_runtime.h>
#include <stdio.h>

__global__ void k_copy(const float4* __restrict__ in, float4* __restrict__ out, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

int main()
{
    const size_t bytes = (size_t)256 << 20;   // 256 MiB read + 256 MiB written per dispatch
    const size_t n = bytes / sizeof(float4);
    float4 *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) return 1;
    if (hipMemset(a, 1, bytes) != hipSuccess) return 1;
    for (int rep = 0; rep < 3; ++rep) hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, 0, a, b, n);
    if (hipDeviceSynchronize() != hipSuccess) return 1;
    printf("copy: %zu bytes read and %zu bytes written per dispatch (%zu KiB each), 3 dispatches\n", bytes, bytes,
           bytes >> 10);
    (void)hipFree(a);
    (void)hipFree(b);
    return 0;
}

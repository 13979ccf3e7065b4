// Standalone building blocks: unfold (Sec. 4.4, Eq. (17)) and a direct FIR
// filter with arbitrary taps (Sec. 4.3, Eq. (15)).
//
// Unfold: Y[i][j] = x[i*stride + j].  A pure gather whose output is
// width/stride times the input; each thread writes 4 consecutive outputs
// (one 16-byte store when a row holds whole groups of 4).
//
// FIR: y[i] = sum_k a[k] x[i-k].  A complex signal is two interleaved float
// streams, so in float indices y[j] = sum_k a[k] x[j - cf*k].  Each 256-thread
// block stages its T = 256*R output floats plus the cf*(K-1) floats of history
// in LDS, then every thread accumulates R outputs spaced 256 apart (so the
// LDS reads of a wave are consecutive); the tap a[k] is the same for the whole
// block at each step and comes through the scalar cache.
#include <stdlib.h>
#include <string.h>

#include <new>
#include <string>

#include "runtime_types.h"
#include "tina_ops.h"

using namespace tina;

namespace {

__global__ __launch_bounds__(256) void unfold_kernel(const float* __restrict__ x, int64_t width, int64_t stride,
                                                     float* __restrict__ y, int64_t total, bool vec) {
    const int64_t n4 = (total + 3) / 4;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n4; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = 4 * t;
        if (vec) {  // width % 4 == 0 and y 16-byte aligned: the 4 outputs share one row
            const int64_t row = e / width, col = e - row * width;
            const float* src = x + row * stride + col;
            *reinterpret_cast<float4*>(y + e) = make_float4(src[0], src[1], src[2], src[3]);
        } else {
            for (int64_t k = e; k < e + 4 && k < total; ++k) {
                const int64_t row = k / width, col = k - row * width;
                y[k] = x[row * stride + col];
            }
        }
    }
}

constexpr int kFirR = 8;                  // outputs per thread
constexpr int kFirT = 256 * kFirR;        // output floats per block

__global__ __launch_bounds__(256) void fir_direct_kernel(const float* __restrict__ x, int64_t nf,
                                                         const float* __restrict__ taps, int K, int cf,
                                                         float* __restrict__ y) {
    extern __shared__ float tile[];       // kFirT + cf*(K-1) floats
    const int64_t halo = (int64_t)cf * (K - 1);
    const int64_t j0 = (int64_t)blockIdx.x * kFirT;
    for (int64_t i = threadIdx.x; i < kFirT + halo; i += 256) {
        const int64_t src = j0 - halo + i;
        tile[i] = (src >= 0 && src < nf) ? x[src] : 0.0f;
    }
    __syncthreads();
    float acc[kFirR];
#pragma unroll
    for (int r = 0; r < kFirR; ++r) acc[r] = 0.0f;
    const float* base = tile + halo + threadIdx.x;
    for (int k = 0; k < K; ++k) {
        const float a = taps[k];
        const float* b = base - cf * k;
#pragma unroll
        for (int r = 0; r < kFirR; ++r) acc[r] = fmaf(a, b[256 * r], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < kFirR; ++r) {
        const int64_t j = j0 + threadIdx.x + 256 * r;
        if (j < nf) y[j] = acc[r];
    }
}

}  // namespace

struct tina_fir_s {
    int device = 0;
    int K = 0, cf = 1;
    float* taps = nullptr;
};

extern "C" {

tina_status tina_unfold(const float* d_x, int64_t n, int64_t width, int64_t stride, float* d_y, int64_t cap,
                        int64_t* rows_out, void* stream) {
    if (n < 0 || width < 1 || stride < 1) return fail(TINA_ERR_INVALID_ARGUMENT, "unfold: need n >= 0, width >= 1, stride >= 1");
    const int64_t rows = n < width ? 0 : (n - width) / stride + 1;
    if (rows > 0 && (!d_x || !d_y)) return fail(TINA_ERR_INVALID_ARGUMENT, "unfold: NULL buffer");
    if (rows > cap) return fail(TINA_ERR_INVALID_ARGUMENT, "unfold: output capacity below " + std::to_string(rows) + " rows");
    if (rows_out) *rows_out = rows;
    if (rows == 0) return TINA_OK;
    const int64_t total = rows * width;
    const bool vec = (width % 4 == 0) && ((uintptr_t)d_y % 16 == 0);
    const int64_t blocks = std::min<int64_t>((total / 4 + 255) / 256 + 1, 1 << 20);
    hipLaunchKernelGGL(unfold_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, d_x, width, stride,
                       d_y, total, vec);
    HIP_TRY(hipGetLastError());
    return TINA_OK;
}

tina_status tina_fir_create(int device, const double* taps, int32_t K, int32_t sample_type, tina_fir_t* out) {
    if (!out || !taps) return fail(TINA_ERR_INVALID_ARGUMENT, "fir_create: NULL argument");
    *out = nullptr;
    if (K < 1 || K > 8192) return fail(TINA_ERR_UNSUPPORTED, "fir_create: taps must be in [1, 8192]");
    if (sample_type != TINA_SAMPLE_R32 && sample_type != TINA_SAMPLE_C64)
        return fail(TINA_ERR_INVALID_ARGUMENT, "fir_create: unknown sample type");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(TINA_ERR_INVALID_ARGUMENT, "fir_create: bad device");
    DeviceScope ds(device);
    tina_fir_s* f = new (std::nothrow) tina_fir_s();
    if (!f) return fail(TINA_ERR_OUT_OF_MEMORY, "fir_create: host allocation");
    f->device = device;
    f->K = K;
    f->cf = sample_type == TINA_SAMPLE_C64 ? 2 : 1;
    float* h = (float*)malloc(sizeof(float) * K);
    if (!h) {
        delete f;
        return fail(TINA_ERR_OUT_OF_MEMORY, "fir_create: host allocation");
    }
    for (int k = 0; k < K; ++k) h[k] = (float)taps[k];
    hipError_t e = hipMalloc(&f->taps, sizeof(float) * K);
    if (e == hipSuccess) e = hipMemcpy(f->taps, h, sizeof(float) * K, hipMemcpyHostToDevice);
    free(h);
    if (e != hipSuccess) {
        if (f->taps) (void)hipFree(f->taps);
        delete f;
        return fail(TINA_ERR_OUT_OF_MEMORY, std::string("fir_create: ") + hipGetErrorString(e));
    }
    const int lds = (int)sizeof(float) * (kFirT + 2 * 8191);
    (void)hipFuncSetAttribute((const void*)fir_direct_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    *out = f;
    return TINA_OK;
}

tina_status tina_fir_destroy(tina_fir_t f) {
    if (!f) return TINA_OK;
    DeviceScope ds(f->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(f->taps);
    delete f;
    return TINA_OK;
}

tina_status tina_fir_execute(tina_fir_t f, const void* d_x, int64_t n, void* d_y, void* stream) {
    if (!f) return fail(TINA_ERR_INVALID_ARGUMENT, "fir_execute: NULL filter");
    if (n < 0) return fail(TINA_ERR_INVALID_ARGUMENT, "fir_execute: negative sample count");
    if (n == 0) return TINA_OK;
    if (!d_x || !d_y) return fail(TINA_ERR_INVALID_ARGUMENT, "fir_execute: NULL buffer");
    const int64_t nf = n * f->cf;
    const uintptr_t xa = (uintptr_t)d_x, ya = (uintptr_t)d_y;
    if (xa % 4 || ya % 4) return fail(TINA_ERR_INVALID_ARGUMENT, "fir_execute: buffers must be 4-byte aligned");
    if (xa < ya + (uintptr_t)nf * 4 && ya < xa + (uintptr_t)nf * 4)
        return fail(TINA_ERR_INVALID_ARGUMENT, "fir_execute: input and output overlap");
    DeviceScope ds(f->device);
    const int64_t blocks = (nf + kFirT - 1) / kFirT;
    const size_t lds = sizeof(float) * (kFirT + (size_t)f->cf * (f->K - 1));
    hipLaunchKernelGGL(fir_direct_kernel, dim3((unsigned)blocks), dim3(256), lds, (hipStream_t)stream,
                       (const float*)d_x, nf, f->taps, f->K, f->cf, (float*)d_y);
    HIP_TRY(hipGetLastError());
    return TINA_OK;
}

}  // extern "C"

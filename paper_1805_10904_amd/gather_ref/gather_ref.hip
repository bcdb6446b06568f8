// Reference gather rate of the device: words[idx[i]] read for i < m over an
// array of n 8-byte words, nothing else.  The sweeps read one published
// word per row entry at a random column; this kernel does only those reads,
// in the same order, so its time is what the memory system gives that
// access pattern with no other work.  Built as a library of its own beside
// the method's; only the measurement harness calls it.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__global__ __launch_bounds__(256) void k_words(uint64_t *words, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) words[i] = (uint64_t)i * 0x9E3779B97F4A7C15ull;
}

// Thread t of workgroup b reads words[idx[i]] for i = b * 256 * PER + t +
// q * 256, q < PER (consecutive threads, consecutive indices), and writes one
// word, the XOR of what it read, so that the output adds 1 / PER of the
// reads' count in stores.
template <int PER>
__global__ __launch_bounds__(256) void k_gather(const uint64_t *__restrict__ words, const int32_t *__restrict__ idx,
                                                uint64_t *__restrict__ out, int64_t m) {
    const int64_t base = (int64_t)blockIdx.x * 256 * PER + threadIdx.x;
    uint64_t v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int64_t i = base + (int64_t)q * 256;
        v[q] = i < m ? words[idx[i]] : 0;
    }
    uint64_t x = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) x ^= v[q];
    if (base < m) out[(int64_t)blockIdx.x * 256 + threadIdx.x] = x;
}

template <int PER>
hipError_t time_gather(const uint64_t *words, const int32_t *idx, uint64_t *out, int64_t m, int reps,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1, float *us) {
    const unsigned nb = (unsigned)((m + 256 * PER - 1) / (256 * PER));
    for (int r = 0; r < 2; ++r) k_gather<PER><<<nb, 256, 0, s>>>(words, idx, out, m);
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) k_gather<PER><<<nb, 256, 0, s>>>(words, idx, out, m);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) e = hipGetLastError();
    *us = ms * 1000.0f / (float)reps;
    return e;
}

}  // namespace

// idx: device int32[m], every value in [0, n) (the caller checks); the
// library allocates the words and the output itself and frees them before
// returning.  *us receives the better of 4 and 16 reads per thread,
// averaged over reps launches on a stream of its own.  Returns a hipError_t.
extern "C" int gather_ref_us(const int32_t *idx, int64_t m, int64_t n, int reps, float *us) {
    if (!idx || m <= 0 || n <= 0 || reps <= 0 || !us) return (int)hipErrorInvalidValue;
    uint64_t *words = nullptr, *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&words, (size_t)n * 8);
    if (e == hipSuccess) e = hipMalloc(&out, (size_t)((m + 1023) / 1024 * 256) * 8);   // one word per thread at PER 4
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        k_words<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(words, n);
        float t4 = 0, t16 = 0;
        e = time_gather<4>(words, idx, out, m, reps, s, e0, e1, &t4);
        if (e == hipSuccess) e = time_gather<16>(words, idx, out, m, reps, s, e0, e1, &t16);
        *us = t4 < t16 ? t4 : t16;
    }
    if (s) (void)hipStreamSynchronize(s);
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (s) (void)hipStreamDestroy(s);
    if (out) (void)hipFree(out);
    if (words) (void)hipFree(words);
    return (int)e;
}

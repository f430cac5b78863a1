// valu_probe.hip -- issue cost of single VALU instruction kinds on gfx950.
//
// A measurement helper for the sweep kernel's roofline (loaded by the
// benchmark, not part of the PTHR library): every work-item runs 8
// independent chains of one instruction, written in inline assembly so the
// compiler cannot change it, and the kernel is launched with far more waves
// than the SIMDs hold.  valu_probe_run returns the elapsed time of `reps`
// launches; cycles per wave64 instruction per SIMD follow from the clock and
// the SIMD count.  No instruction here touches memory except the final store
// of one word per work-item.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kIters = 1024;
constexpr int kChains = 8;
constexpr int kThreads = 256;

#define PROBE_LOOP(BODY)                                       \
  for (int it = 0; it < kIters; ++it) {                        \
    _Pragma("unroll") for (int c = 0; c < kChains; ++c) {      \
      BODY;                                                    \
    }                                                          \
  }

template <int KIND>
__global__ __launch_bounds__(kThreads) void probe_kernel(uint32_t* out, uint32_t seed) {
  uint32_t v[kChains];
  double d[kChains];
  uint64_t m[kChains];
  for (int c = 0; c < kChains; ++c) {
    v[c] = seed + threadIdx.x * 7u + c * 13u;
    d[c] = static_cast<double>(v[c] & 1023u) * 1e-3;
    m[c] = 0x5555555555555555ull * static_cast<uint64_t>(c + 1);
  }
  const uint32_t a = seed | 1u, b = seed ^ 0x5555u;
  const float fa = 1.0000001f;
  const double da = 1.0000001;
  if constexpr (KIND == 0) PROBE_LOOP(asm volatile("v_add_f32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 1) PROBE_LOOP(asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(v[c]) : "v"(fa), "v"(b)))
  if constexpr (KIND == 2) PROBE_LOOP(asm volatile("v_xor_b32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 3) PROBE_LOOP(asm volatile("v_add_u32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 4) PROBE_LOOP(asm volatile("v_ashrrev_i32 %0, %1, %0" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 5) PROBE_LOOP(asm volatile("v_lshlrev_b32 %0, %1, %0" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 6) PROBE_LOOP(asm volatile("v_bfi_b32 %0, %0, %1, %2" : "+v"(v[c]) : "v"(a), "v"(b)))
  if constexpr (KIND == 7) PROBE_LOOP(asm volatile("v_and_or_b32 %0, %0, %1, %2" : "+v"(v[c]) : "v"(a), "v"(b)))
  if constexpr (KIND == 8) PROBE_LOOP(asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(v[c]) : "v"(a), "s"(b)))
  if constexpr (KIND == 9) PROBE_LOOP({
    uint64_t r;
    asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(r) : "v"(v[c]), "v"(a) : "vcc");
    v[c] = static_cast<uint32_t>(r >> 32);
  })
  if constexpr (KIND == 10) PROBE_LOOP(asm volatile("v_cvt_f32_u32 %0, %0" : "+v"(v[c])))
  if constexpr (KIND == 11) PROBE_LOOP(asm volatile("v_rndne_f32 %0, %0" : "+v"(v[c])))
  if constexpr (KIND == 12) PROBE_LOOP(asm volatile("v_ldexp_f32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 13) PROBE_LOOP(asm volatile("v_cmp_le_f32_e64 %0, %1, %2" : "+s"(m[c]) : "v"(v[c]), "v"(a)))
  if constexpr (KIND == 14) PROBE_LOOP(asm volatile("v_alignbit_b32 %0, %0, %1, 31" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 15) PROBE_LOOP(asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(d[c]) : "v"(da)))
  if constexpr (KIND == 16) PROBE_LOOP(asm volatile("v_add_f64 %0, %0, %1" : "+v"(d[c]) : "v"(da)))
  if constexpr (KIND == 17) PROBE_LOOP(asm volatile("v_exp_f32 %0, %0" : "+v"(v[c])))
  if constexpr (KIND == 18) PROBE_LOOP(asm volatile("v_sub_f32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 19) PROBE_LOOP(asm volatile("v_mul_f32_e64 %0, -%0, %1" : "+v"(v[c]) : "v"(fa)))
  if constexpr (KIND == 20) PROBE_LOOP(asm volatile("v_fmaak_f32 %0, %0, %1, 0x3f000000" : "+v"(v[c]) : "v"(fa)))
  if constexpr (KIND == 21) PROBE_LOOP(asm volatile("v_and_b32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 22) PROBE_LOOP(asm volatile("v_or_b32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 23) PROBE_LOOP(asm volatile("v_sub_u32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 24) PROBE_LOOP(asm volatile("v_lshrrev_b32 %0, %1, %0" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 25) PROBE_LOOP(asm volatile("v_mov_b32 %0, %1" : "=v"(v[c]) : "v"(v[(c + 1) % kChains])))
  if constexpr (KIND == 26) PROBE_LOOP(asm volatile("v_bfe_i32 %0, %0, %1, 1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 27) PROBE_LOOP(asm volatile("v_max_f32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 28) PROBE_LOOP(asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(v[c]) : "v"(a), "v"(b)))
  if constexpr (KIND == 29) PROBE_LOOP(asm volatile("v_lshl_add_u32 %0, %0, 3, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 30) PROBE_LOOP(asm volatile("v_perm_b32 %0, %0, %1, %2" : "+v"(v[c]) : "v"(a), "v"(b)))
  if constexpr (KIND == 31) PROBE_LOOP(asm volatile("v_cvt_i32_f32 %0, %0" : "+v"(v[c])))
  if constexpr (KIND == 32) PROBE_LOOP(asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 33) PROBE_LOOP(asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 34) PROBE_LOOP({
    uint64_t co;
    asm volatile("v_addc_co_u32_e64 %0, %1, %0, %0, %2" : "+v"(v[c]), "=s"(co) : "s"(m[0]));
  })
  if constexpr (KIND == 35) PROBE_LOOP(asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(v[c]) : "v"(a), "s"(m[0])))
  if constexpr (KIND == 36) PROBE_LOOP(asm volatile("v_mul_f64 %0, %0, %1" : "+v"(d[c]) : "v"(da)))
  if constexpr (KIND == 37) PROBE_LOOP(asm volatile("v_ldexp_f64 %0, %0, %1" : "+v"(d[c]) : "v"(a)))
  if constexpr (KIND == 38) PROBE_LOOP(asm volatile("v_rndne_f64 %0, %0" : "+v"(d[c])))
  if constexpr (KIND == 39) PROBE_LOOP(asm volatile("v_cvt_f64_u32 %0, %1" : "=v"(d[c]) : "v"(v[c])))
  if constexpr (KIND == 40) PROBE_LOOP(asm volatile("v_cmp_lt_f64_e64 %0, %1, %2" : "+s"(m[c]) : "v"(d[c]), "v"(da)))
  if constexpr (KIND == 41) PROBE_LOOP(asm volatile("v_lshlrev_b64 %0, 1, %0" : "+v"(m[c])))
  if constexpr (KIND == 42) PROBE_LOOP(asm volatile("v_lshl_add_u64 %0, %0, 1, %1" : "+v"(m[c]) : "v"(m[(c + 1) % kChains])))
  if constexpr (KIND == 43) PROBE_LOOP(asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(v[c]) : "v"(a)))
  if constexpr (KIND == 44) PROBE_LOOP(asm volatile("v_lshl_or_b32 %0, %0, 1, %1" : "+v"(v[c]) : "v"(a)))
  uint32_t acc = 0;
  for (int c = 0; c < kChains; ++c)
    acc ^= v[c] ^ static_cast<uint32_t>(__double_as_longlong(d[c])) ^ static_cast<uint32_t>(m[c]);
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

const char* const kNames[] = {"v_add_f32",     "v_fma_f32",     "v_xor_b32",    "v_add_u32",        "v_ashrrev_i32",
                              "v_lshlrev_b32", "v_bfi_b32",     "v_and_or_b32", "v_bitop3_b32",     "v_mad_u64_u32",
                              "v_cvt_f32_u32", "v_rndne_f32",   "v_ldexp_f32",  "v_cmp_le_f32_e64", "v_alignbit_b32",
                              "v_fma_f64",     "v_add_f64",     "v_exp_f32",    "v_sub_f32",        "v_mul_f32_e64_neg",
                              "v_fmaak_f32",   "v_and_b32",     "v_or_b32",     "v_sub_u32",        "v_lshrrev_b32",
                              "v_mov_b32",     "v_bfe_i32",     "v_max_f32",    "v_add3_u32",       "v_lshl_add_u32",
                              "v_perm_b32",    "v_cvt_i32_f32", "v_mul_lo_u32", "v_mul_hi_u32",     "v_addc_co_u32_e64",
                              "v_cndmask_b32_e64", "v_mul_f64", "v_ldexp_f64",  "v_rndne_f64",      "v_cvt_f64_u32",
                              "v_cmp_lt_f64_e64", "v_lshlrev_b64", "v_lshl_add_u64", "v_pk_add_u16", "v_lshl_or_b32"};
constexpr int kKinds = sizeof(kNames) / sizeof(kNames[0]);

template <int KIND>
hipError_t launch(int blocks, uint32_t* out, uint32_t seed) {
  hipLaunchKernelGGL(probe_kernel<KIND>, dim3(blocks), dim3(kThreads), 0, 0, out, seed);
  return hipGetLastError();
}

template <int... K>
hipError_t dispatch(int kind, int blocks, uint32_t* out, uint32_t seed, std::integer_sequence<int, K...>) {
  hipError_t e = hipErrorInvalidValue;
  ((kind == K ? (e = launch<K>(blocks, out, seed), 0) : 0), ...);
  return e;
}

}  // namespace

extern "C" {

// Number of instruction kinds and the name of kind k (NULL if out of range).
int valu_probe_kinds(void) { return kKinds; }
const char* valu_probe_name(int k) { return k >= 0 && k < kKinds ? kNames[k] : nullptr; }

// Times `reps` launches of `blocks` workgroups of 256 work-items running kind
// k (after one untimed launch) on the default stream.  *ms: elapsed time;
// *wave_instructions: wave64 instructions of the probed kind executed in the
// timed launches.  0 on success, -1 on a bad argument, -3 on a HIP error.
int valu_probe_run(int k, int blocks, int reps, double* ms, double* wave_instructions) {
  if (k < 0 || k >= kKinds || blocks < 1 || reps < 1 || !ms || !wave_instructions) return -1;
  uint32_t* out = nullptr;
  if (hipMalloc(&out, sizeof(uint32_t) * size_t(blocks) * kThreads) != hipSuccess) return -3;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0;
  auto seq = std::make_integer_sequence<int, kKinds>{};
  float t = 0.f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -3;
  if (rc == 0 && dispatch(k, blocks, out, 12345u, seq) != hipSuccess) rc = -3;
  if (rc == 0 && hipEventRecord(e0, nullptr) != hipSuccess) rc = -3;
  for (int r = 0; rc == 0 && r < reps; ++r)
    if (dispatch(k, blocks, out, 12345u + r, seq) != hipSuccess) rc = -3;
  if (rc == 0 && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    rc = -3;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (rc == 0) {
    *ms = t;
    *wave_instructions = double(reps) * blocks * (kThreads / 64) * double(kIters) * kChains;
  }
  return rc;
}

}  // extern "C"

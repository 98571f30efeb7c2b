// Issue cost of the VALU instruction forms the traversal kernels are made of,
// measured on the device: one workgroup on one CU runs `waves_per_simd` waves
// on each of its four SIMDs, each wave issuing `iters` rounds of twelve
// independent instructions of one form (written in inline assembly, so the
// form is exactly the one named). The cycles per wave64 instruction per SIMD
// follow from the launch time. One CU, because with every CU running dense
// VALU code the chip lowers its clock to stay within its power limit, and the
// figure would then measure that limit instead of the instruction. The
// instruction ceiling of a kernel is its counted mix of these forms. This is a
// measurement aid for the benchmark, not part of the library's interface
// (libwfpg_probe.so, no header).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 12;

enum {
    OP_ADD_E32 = 0,        // v_add_u32_e32      two VGPR operands (VOP2)
    OP_XOR_E32,            // v_xor_b32_e32
    OP_CNDMASK_E64,        // v_cndmask_b32_e64  select on a lane mask in an SGPR pair
    OP_CMP_E64,            // v_cmp_eq_u32_e64   32-bit compare into an SGPR pair
    OP_CMP64_E64,          // v_cmp_gt_u64_e64   64-bit compare into an SGPR pair
    OP_MAD_U64,            // v_mad_u64_u32      32 x 32 + 64 -> 64
    OP_LSHL_ADD_U64,       // v_lshl_add_u64     64-bit add
    OP_BITOP3,             // v_bitop3_b32       three-operand 32-bit logic
    OP_LSHL_E64,           // v_lshlrev_b32_e64  two-operand op in the three-operand encoding
    OP_COUNT
};

template <int OP>
__global__ void __launch_bounds__(1024) k_issue(uint32_t *out, int iters, uint64_t lane_mask)
{
    uint32_t x[kChains];
    uint64_t m[kChains], sg[kChains];   // sg: scalar results, read once after the loop
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        x[c] = threadIdx.x * 0x9E3779B9u + (uint32_t)c * 7u + 1u;
        m[c] = ((uint64_t)x[c] << 21) ^ x[c];
        sg[c] = 0;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            const int d = (c + 1) % kChains;
            if constexpr (OP == OP_ADD_E32) {
                asm volatile("v_add_u32_e32 %0, %1, %0" : "+v"(x[c]) : "v"(x[d]));
            } else if constexpr (OP == OP_XOR_E32) {
                asm volatile("v_xor_b32_e32 %0, %1, %0" : "+v"(x[c]) : "v"(x[d]));
            } else if constexpr (OP == OP_CNDMASK_E64) {
                asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(x[c]) : "v"(x[d]), "s"(lane_mask));
            } else if constexpr (OP == OP_CMP_E64) {
                asm volatile("v_cmp_eq_u32_e64 %0, %1, %2" : "=s"(sg[c]) : "v"(x[c]), "v"(x[d]));
            } else if constexpr (OP == OP_CMP64_E64) {
                asm volatile("v_cmp_gt_u64_e64 %0, %1, %2" : "=s"(sg[c]) : "v"(m[c]), "v"(m[d]));
            } else if constexpr (OP == OP_MAD_U64) {
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(m[c]), "=s"(sg[c]) : "v"(x[c]), "v"(x[d]));
            } else if constexpr (OP == OP_LSHL_ADD_U64) {
                asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(m[c]) : "v"(m[d]));
            } else if constexpr (OP == OP_BITOP3) {
                asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(x[c]) : "v"(x[d]), "v"(x[(c + 2) % kChains]));
            } else {
                asm volatile("v_lshlrev_b32_e64 %0, %1, %0" : "+v"(x[c]) : "v"(x[d]));
            }
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) r ^= x[c] ^ (uint32_t)m[c] ^ (uint32_t)(m[c] >> 32) ^ (uint32_t)sg[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

template <int OP>
void launch(uint32_t *out, int threads, int iters, hipStream_t st)
{
    hipLaunchKernelGGL(k_issue<OP>, dim3(1), dim3(threads), 0, st, out, iters, 0x5555555555555555ull);
}

void launch_op(int op, uint32_t *out, int threads, int iters, hipStream_t st)
{
    switch (op) {
    case OP_ADD_E32: launch<OP_ADD_E32>(out, threads, iters, st); break;
    case OP_XOR_E32: launch<OP_XOR_E32>(out, threads, iters, st); break;
    case OP_CNDMASK_E64: launch<OP_CNDMASK_E64>(out, threads, iters, st); break;
    case OP_CMP_E64: launch<OP_CMP_E64>(out, threads, iters, st); break;
    case OP_CMP64_E64: launch<OP_CMP64_E64>(out, threads, iters, st); break;
    case OP_MAD_U64: launch<OP_MAD_U64>(out, threads, iters, st); break;
    case OP_LSHL_ADD_U64: launch<OP_LSHL_ADD_U64>(out, threads, iters, st); break;
    case OP_BITOP3: launch<OP_BITOP3>(out, threads, iters, st); break;
    default: launch<OP_LSHL_E64>(out, threads, iters, st); break;
    }
}

}  // namespace

// Number of instruction forms the probe measures (op = 0 .. count - 1).
extern "C" int wfpg_probe_valu_forms(void)
{
    return OP_COUNT;
}

// Time one launch of form `op` on the current device: one workgroup of
// 4 x waves_per_simd (1..4) waves, waves_per_simd on each SIMD of one CU, each
// issuing iters x 12 instructions of that form. *ms receives the launch time
// (HIP events on the null stream, after one untimed launch) and
// *instr_per_simd the wave instructions each SIMD issued. Returns a hipError_t
// (hipErrorInvalidValue for arguments out of range). Synchronizes the device.
extern "C" int wfpg_probe_valu_issue(int op, int waves_per_simd, int iters, float *ms, double *instr_per_simd)
{
    if (op < 0 || op >= OP_COUNT || waves_per_simd < 1 || waves_per_simd > 4 || iters < 1 || !ms ||
        !instr_per_simd)
        return hipErrorInvalidValue;
    const int threads = 256 * waves_per_simd;
    uint32_t *out = nullptr;
    hipError_t e = hipMalloc(&out, (size_t)threads * sizeof(uint32_t));
    if (e != hipSuccess) return e;
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) {
        launch_op(op, out, threads, iters, 0);
        e = hipEventRecord(a, 0);
    }
    if (e == hipSuccess) {
        launch_op(op, out, threads, iters, 0);
        e = hipEventRecord(b, 0);
    }
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    if (e == hipSuccess) e = hipGetLastError();
    *instr_per_simd = (double)waves_per_simd * iters * kChains;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    const hipError_t ef = hipFree(out);
    return e != hipSuccess ? e : ef;
}

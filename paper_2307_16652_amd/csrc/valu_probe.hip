// valu_probe.hip -- measures how fast the vector unit of gfx950 issues the
// instruction classes the PaLD kernels are built from (libpald_probe.so).
//
// Measurement support for the roofline, not part of the method: every probe
// kernel runs a long loop of independent register-only instructions of one
// class (or a fixed mix) in every wave of a full grid, with no memory access
// inside the loop, and reports SIMD cycles per wave64 instruction: the kernel
// time (HIP events) times the shader clock (memtime ticks over the 100 MHz
// real-time counter, read by every wave around its loop) times the SIMD count,
// divided by the wave instructions issued.  A class that issues once per four
// cycles (16 lanes a cycle) reads 4; one that issues twice as often reads 2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "pairwise.hpp"
#include "triplet.hpp"

namespace {

#define PQ_R8(I) I(0) I(1) I(2) I(3) I(4) I(5) I(6) I(7)
#define PQ_R16(I) PQ_R8(I) I(8) I(9) I(10) I(11) I(12) I(13) I(14) I(15)
#define PQ_R32(I) PQ_R16(I) PQ_R16(I)
// one instruction on register a<k> (16 independent chains)
#define PQ_ADDF(k) "v_add_f32 %[a" #k "], %[a" #k "], %[b]\n\t"
#define PQ_FMAF(k) "v_fma_f32 %[a" #k "], %[a" #k "], %[b], %[c]\n\t"
#define PQ_ADDU(k) "v_add_u32 %[a" #k "], %[a" #k "], %[b]\n\t"
#define PQ_ANDB(k) "v_and_b32 %[a" #k "], %[a" #k "], %[b]\n\t"
#define PQ_MINU(k) "v_min_u32 %[a" #k "], %[a" #k "], %[b]\n\t"
#define PQ_MINF(k) "v_min_f32 %[a" #k "], %[a" #k "], %[b]\n\t"
#define PQ_CMPU(k) "v_cmp_lt_u32_e64 %[s" #k "], %[a" #k "], %[b]\n\t"
#define PQ_CMPF(k) "v_cmp_le_f32_e64 %[s" #k "], %[a" #k "], %[b]\n\t"
#define PQ_CND(k) "v_cndmask_b32_e64 %[a" #k "], %[a" #k "], %[b], %[m]\n\t"
#define PQ_ADDC(k) "v_addc_co_u32_e64 %[a" #k "], %[co], 0, %[a" #k "], %[m]\n\t"
#define PQ_CMPU_ADDF(k) "v_cmp_lt_u32_e64 %[s" #k "], %[a" #k "], %[b]\n\tv_add_f32 %[f" #k "], %[f" #k "], %[c]\n\t"
#define PQ_MINU_ADDF(k) "v_min_u32 %[a" #k "], %[a" #k "], %[b]\n\tv_add_f32 %[f" #k "], %[f" #k "], %[c]\n\t"
#define PQ_MINU_ANDB(k) "v_min_u32 %[a" #k "], %[a" #k "], %[b]\n\tv_and_b32 %[f" #k "], %[f" #k "], %[c]\n\t"
#define PQ_PKSUB(k) "v_pk_sub_i16 %[a" #k "], %[a" #k "], %[b]\n\t"
#define PQ_PKMIN(k) "v_pk_min_i16 %[a" #k "], %[a" #k "], %[b]\n\t"
#define PQ_PKSHR(k) "v_pk_lshrrev_b16 %[a" #k "], 15, %[a" #k "]\n\t"
#define PQ_PKADD(k) "v_pk_add_u16 %[a" #k "], %[a" #k "], %[b]\n\t"

#define PQ_AOUT(k) [a##k] "+v"(a[k])
#define PQ_FOUT(k) [f##k] "+v"(f[k])
#define PQ_SOUT(k) [s##k] "=&s"(s[k])
#define PQ_AOUT16 PQ_AOUT(0), PQ_AOUT(1), PQ_AOUT(2), PQ_AOUT(3), PQ_AOUT(4), PQ_AOUT(5), PQ_AOUT(6), PQ_AOUT(7), \
    PQ_AOUT(8), PQ_AOUT(9), PQ_AOUT(10), PQ_AOUT(11), PQ_AOUT(12), PQ_AOUT(13), PQ_AOUT(14), PQ_AOUT(15)
#define PQ_FOUT16 PQ_FOUT(0), PQ_FOUT(1), PQ_FOUT(2), PQ_FOUT(3), PQ_FOUT(4), PQ_FOUT(5), PQ_FOUT(6), PQ_FOUT(7), \
    PQ_FOUT(8), PQ_FOUT(9), PQ_FOUT(10), PQ_FOUT(11), PQ_FOUT(12), PQ_FOUT(13), PQ_FOUT(14), PQ_FOUT(15)
#define PQ_AIN(k) [a##k] "v"(a[k])
#define PQ_AIN16 PQ_AIN(0), PQ_AIN(1), PQ_AIN(2), PQ_AIN(3), PQ_AIN(4), PQ_AIN(5), PQ_AIN(6), PQ_AIN(7), PQ_AIN(8), \
    PQ_AIN(9), PQ_AIN(10), PQ_AIN(11), PQ_AIN(12), PQ_AIN(13), PQ_AIN(14), PQ_AIN(15)
#define PQ_SOUT16 PQ_SOUT(0), PQ_SOUT(1), PQ_SOUT(2), PQ_SOUT(3), PQ_SOUT(4), PQ_SOUT(5), PQ_SOUT(6), PQ_SOUT(7), \
    PQ_SOUT(8), PQ_SOUT(9), PQ_SOUT(10), PQ_SOUT(11), PQ_SOUT(12), PQ_SOUT(13), PQ_SOUT(14), PQ_SOUT(15)

// Probe classes and their vector instructions per loop iteration.
enum {
    PQ_C_ADD_F32 = 0, PQ_C_FMA_F32, PQ_C_ADD_U32, PQ_C_AND_B32, PQ_C_MIN_U32, PQ_C_MIN_F32, PQ_C_CMP_U32, PQ_C_CMP_F32,
    PQ_C_CNDMASK, PQ_C_ADDC, PQ_C_CMP_AND_ADD_F32, PQ_C_MIN_AND_ADD_F32, PQ_C_MIN_AND_AND_B32, PQ_C_COHESION_BLOCK,
    PQ_C_TRIPLET_BLOCK, PQ_C_PK_SUB_I16, PQ_C_PK_MIN_I16, PQ_C_PK_LSHR_B16, PQ_C_PK_ADD_U16, PQ_C_RANK_BLOCK,
    PQ_NUM_CLASSES
};
constexpr int kInstrPerIter[PQ_NUM_CLASSES] = {32, 32, 32, 32, 32, 32, 32, 32, 32, 32, 64, 64, 64, 32, 52,
                                                32, 32, 32, 32, 40};

template <int CLS>
__global__ __launch_bounds__(256) void probe_kernel(uint64_t *__restrict__ stamps, uint32_t *__restrict__ sink,
                                                    int32_t iters, uint64_t mask) {
    uint32_t a[16], f[16];
    for (int k = 0; k < 16; ++k) {
        a[k] = __float_as_uint(1.0f + (float)threadIdx.x * 1e-3f + (float)k);
        f[k] = a[k] ^ 0x1u;
    }
    const uint32_t b = __float_as_uint(1e-7f) ^ (threadIdx.x & 1u), c = __float_as_uint(0.5f);
    uint64_t s[16] = {};
    uint64_t co = 0;
    const uint64_t m = mask;
    const uint64_t full = __builtin_amdgcn_read_exec();
    __syncthreads();
    const uint64_t t0 = clock64(), r0 = wall_clock64();
    for (int32_t it = 0; it < iters; ++it) {
        if constexpr (CLS == PQ_C_ADD_F32) asm volatile(PQ_R32(PQ_ADDF) : PQ_AOUT16 : [b] "v"(b));
        if constexpr (CLS == PQ_C_FMA_F32) asm volatile(PQ_R32(PQ_FMAF) : PQ_AOUT16 : [b] "v"(b), [c] "v"(c));
        if constexpr (CLS == PQ_C_ADD_U32) asm volatile(PQ_R32(PQ_ADDU) : PQ_AOUT16 : [b] "v"(b));
        if constexpr (CLS == PQ_C_AND_B32) asm volatile(PQ_R32(PQ_ANDB) : PQ_AOUT16 : [b] "v"(b));
        if constexpr (CLS == PQ_C_MIN_U32) asm volatile(PQ_R32(PQ_MINU) : PQ_AOUT16 : [b] "v"(b));
        if constexpr (CLS == PQ_C_MIN_F32) asm volatile(PQ_R32(PQ_MINF) : PQ_AOUT16 : [b] "v"(b));
        if constexpr (CLS == PQ_C_CMP_U32) asm volatile(PQ_R32(PQ_CMPU) : PQ_SOUT16 : PQ_AIN16, [b] "v"(b));
        if constexpr (CLS == PQ_C_CMP_F32) asm volatile(PQ_R32(PQ_CMPF) : PQ_SOUT16 : PQ_AIN16, [b] "v"(b));
        if constexpr (CLS == PQ_C_CNDMASK) asm volatile(PQ_R32(PQ_CND) : PQ_AOUT16 : [b] "v"(b), [m] "s"(m));
        if constexpr (CLS == PQ_C_ADDC) asm volatile(PQ_R32(PQ_ADDC) : PQ_AOUT16, [co] "=&s"(co) : [m] "s"(m));
        if constexpr (CLS == PQ_C_CMP_AND_ADD_F32)
            asm volatile(PQ_R32(PQ_CMPU_ADDF) : PQ_SOUT16, PQ_FOUT16 : PQ_AIN16, [b] "v"(b), [c] "v"(c));
        if constexpr (CLS == PQ_C_MIN_AND_ADD_F32)
            asm volatile(PQ_R32(PQ_MINU_ADDF) : PQ_AOUT16, PQ_FOUT16 : [b] "v"(b), [c] "v"(c));
        if constexpr (CLS == PQ_C_MIN_AND_AND_B32)
            asm volatile(PQ_R32(PQ_MINU_ANDB) : PQ_AOUT16, PQ_FOUT16 : [b] "v"(b), [c] "v"(c));
        if constexpr (CLS == PQ_C_PK_SUB_I16) asm volatile(PQ_R32(PQ_PKSUB) : PQ_AOUT16 : [b] "v"(b));
        if constexpr (CLS == PQ_C_PK_MIN_I16) asm volatile(PQ_R32(PQ_PKMIN) : PQ_AOUT16 : [b] "v"(b));
        if constexpr (CLS == PQ_C_PK_LSHR_B16) asm volatile(PQ_R32(PQ_PKSHR) : PQ_AOUT16);
        if constexpr (CLS == PQ_C_PK_ADD_U16) asm volatile(PQ_R32(PQ_PKADD) : PQ_AOUT16 : [b] "v"(b));
        if constexpr (CLS == PQ_C_RANK_BLOCK) {
            // the rank-form pass-1 block for 16 pairs (8 packed pairs of pairs): per
            // pair of pairs two packed differences (x side, y side with its low half
            // used twice), their packed minimum, its sign bits and a packed count
            uint32_t t[8], u[8];
            asm volatile(
#define PQ_RK1(k) "v_pk_sub_i16 %[t" #k "], %[x" #k "], %[sa]\n\t"
#define PQ_RK2(k) "v_pk_sub_i16 %[u" #k "], %[y], %[sb] op_sel_hi:[0,1]\n\t"
#define PQ_RK3(k) "v_pk_min_i16 %[t" #k "], %[t" #k "], %[u" #k "]\n\t"
#define PQ_RK4(k) "v_pk_lshrrev_b16 %[t" #k "], 15, %[t" #k "]\n\t"
#define PQ_RK5(k) "v_pk_add_u16 %[a" #k "], %[a" #k "], %[t" #k "]\n\t"
                PQ_R8(PQ_RK1) PQ_R8(PQ_RK2) PQ_R8(PQ_RK3) PQ_R8(PQ_RK4) PQ_R8(PQ_RK5)
#undef PQ_RK1
#undef PQ_RK2
#undef PQ_RK3
#undef PQ_RK4
#undef PQ_RK5
                : [a0] "+v"(a[0]), [a1] "+v"(a[1]), [a2] "+v"(a[2]), [a3] "+v"(a[3]), [a4] "+v"(a[4]),
                  [a5] "+v"(a[5]), [a6] "+v"(a[6]), [a7] "+v"(a[7]), [t0] "=&v"(t[0]), [t1] "=&v"(t[1]),
                  [t2] "=&v"(t[2]), [t3] "=&v"(t[3]), [t4] "=&v"(t[4]), [t5] "=&v"(t[5]), [t6] "=&v"(t[6]),
                  [t7] "=&v"(t[7]), [u0] "=&v"(u[0]), [u1] "=&v"(u[1]), [u2] "=&v"(u[2]), [u3] "=&v"(u[3]),
                  [u4] "=&v"(u[4]), [u5] "=&v"(u[5]), [u6] "=&v"(u[6]), [u7] "=&v"(u[7])
                : [x0] "v"(f[0]), [x1] "v"(f[1]), [x2] "v"(f[2]), [x3] "v"(f[3]), [x4] "v"(f[4]), [x5] "v"(f[5]),
                  [x6] "v"(f[6]), [x7] "v"(f[7]), [y] "v"(f[8]), [sa] "s"((uint32_t)m), [sb] "s"((uint32_t)(m >> 32)));
        }
        if constexpr (CLS == PQ_C_COHESION_BLOCK) {
            // the pass-2 block: one x, four z, one y -- 16 compares and 16 masked additions
            float rf[4], rr[4], hz[4];
            uint32_t t[4], bb[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                rf[k] = __uint_as_float(f[k]);
                rr[k] = __uint_as_float(f[k + 4]);
                t[k] = a[k];
                bb[k] = a[k + 4];
                hz[k] = __uint_as_float(c);
            }
            pald::cohesion_terms4<4>(rf, rr, t, a[8], bb, __uint_as_float(b), hz, full);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                f[k] = __float_as_uint(rf[k]);
                f[k + 4] = __float_as_uint(rr[k]);
            }
        }
        if constexpr (CLS == PQ_C_TRIPLET_BLOCK) {
            // the triplet pass-2 block: one p, one q, four r -- per triple a min, three compares, three
            // selects and six multiply-adds under EXEC masks (52 vector instructions)
            float tpq = __uint_as_float(f[12]), tqp = __uint_as_float(f[13]);
            float rf[4], rr[4], tqr[4], trq[4], hpr[4], hc[4];
            uint32_t bb[4], cc[4];
            const uint64_t vr[4] = {full, full, full, full};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                rf[k] = __uint_as_float(f[k]);
                rr[k] = __uint_as_float(f[k + 4]);
                tqr[k] = __uint_as_float(f[k + 8]);
                trq[k] = __uint_as_float(a[k + 12]);
                bb[k] = a[k];
                cc[k] = a[k + 4];
                hpr[k] = __uint_as_float(c);
                hc[k] = __uint_as_float(b);
            }
            pald::triplet_cohesion4(tpq, tqp, rf, rr, tqr, trq, a[8], __uint_as_float(c), bb, hpr, cc, hc, full, vr,
                                    full);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                f[k] = __float_as_uint(rf[k]);
                f[k + 4] = __float_as_uint(rr[k]);
                f[k + 8] = __float_as_uint(tqr[k]);
                a[k + 12] = __float_as_uint(trq[k]);
            }
            f[12] = __float_as_uint(tpq);
            f[13] = __float_as_uint(tqp);
        }
    }
    const uint64_t t1 = clock64(), r1 = wall_clock64();
    const int wave = (int)(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
    uint32_t acc = (uint32_t)co;
    for (int k = 0; k < 16; ++k) acc ^= a[k] ^ f[k] ^ (uint32_t)s[k];
    if ((threadIdx.x & 63) == 0) {
        stamps[4 * wave + 0] = t0;
        stamps[4 * wave + 1] = t1;
        stamps[4 * wave + 2] = r0;
        stamps[4 * wave + 3] = r1;
    }
    sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

typedef void (*ProbeFn)(uint64_t *, uint32_t *, int32_t, uint64_t);
const ProbeFn kProbes[PQ_NUM_CLASSES] = {
    probe_kernel<0>, probe_kernel<1>, probe_kernel<2>, probe_kernel<3>,  probe_kernel<4>,
    probe_kernel<5>, probe_kernel<6>, probe_kernel<7>, probe_kernel<8>,  probe_kernel<9>,
    probe_kernel<10>, probe_kernel<11>, probe_kernel<12>, probe_kernel<13>, probe_kernel<14>,
    probe_kernel<15>, probe_kernel<16>, probe_kernel<17>, probe_kernel<18>, probe_kernel<19>};

}  // namespace

extern "C" {

// Number of probe classes.
int32_t pald_probe_classes(void) { return PQ_NUM_CLASSES; }

// Runs class `cls` with waves_per_simd waves on every SIMD of device 0's
// current device (one workgroup of 4 waves per CU per unit), `iters` loop
// iterations per wave, and writes: out[0] SIMD cycles per wave64 vector
// instruction, out[1] the shader clock in GHz measured around the loops,
// out[2] the kernel time in ms, out[3] vector instructions per iteration.
// Synchronous; allocates and frees its own small buffers.  Returns 0 on
// success, -1 on a bad argument, -2 on a HIP error.
int32_t pald_probe_valu(int32_t cls, int32_t waves_per_simd, int32_t iters, double *out) {
    if (cls < 0 || cls >= PQ_NUM_CLASSES || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || !out) return -1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return -2;
    const int blocks = cus * waves_per_simd;
    uint64_t *stamps = nullptr;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int32_t rc = 0;
    std::vector<uint64_t> h((size_t)blocks * 4 * 4);
    float ms = 0.0f;
    if (hipMalloc(&stamps, h.size() * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&sink, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = -2;
    } else {
        const uint64_t mask = 0x5555555555555555ull;
        kProbes[cls]<<<blocks, 256>>>(stamps, sink, std::max(1, iters / 10), mask);  // warm-up
        (void)hipEventRecord(e0, nullptr);
        kProbes[cls]<<<blocks, 256>>>(stamps, sink, iters, mask);
        (void)hipEventRecord(e1, nullptr);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
            hipMemcpy(h.data(), stamps, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
            rc = -2;
    }
    if (rc == 0) {
        double cyc = 0.0, rt = 0.0;
        for (int w = 0; w < blocks * 4; ++w) {
            cyc += (double)(h[4 * w + 1] - h[4 * w + 0]);
            rt += (double)(h[4 * w + 3] - h[4 * w + 2]);
        }
        const double clk_hz = rt > 0.0 ? cyc / (rt / 100e6) : 0.0;  // the real-time counter runs at 100 MHz
        const double instr = (double)blocks * 4 * iters * kInstrPerIter[cls];
        out[0] = (double)ms * 1e-3 * clk_hz * cus * 4.0 / instr;
        out[1] = clk_hz / 1e9;
        out[2] = (double)ms;
        out[3] = (double)kInstrPerIter[cls];
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (stamps) (void)hipFree(stamps);
    if (sink) (void)hipFree(sink);
    return rc;
}

}  // extern "C"

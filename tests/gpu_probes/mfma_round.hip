// How the 16x16x32 bf16 MFMA of gfx950 rounds its FP32 result: one wave per
// case, row 0 of A and column 0 of B set, every other entry zero, and the
// (0,0) element compared with the exactly rounded (round to nearest even)
// value of the exact sum.  Prints one line per case.  Grid: one block of 64
// threads per case; every lane writes its 4 accumulator values to
// out[case*256 + lane*4 + r], inside the NCASE*256 floats allocated.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstring>
#include <cmath>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int NCASE = 8;

__global__ void probe(const float *av, const float *bv, const float *c00, float *out) {
    const int cs = blockIdx.x, lane = threadIdx.x;
    bf16x8 a, b;
    for (int v = 0; v < 8; ++v) {
        const int k = 8 * (lane >> 4) + v;
        const bool row0 = (lane & 15) == 0;
        a[v] = (__bf16)(row0 ? av[cs * 32 + k] : 0.0f);
        b[v] = (__bf16)(row0 ? bv[cs * 32 + k] : 0.0f);
    }
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    if (lane == 0) acc[0] = c00[cs];
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[cs * 256 + lane * 4 + r] = acc[r];
}

int main() {
    float av[NCASE * 32] = {}, bv[NCASE * 32] = {}, c00[NCASE] = {};
    const char *name[NCASE];
    double exact[NCASE];
    auto set = [&](int cs, int k, float a, float b) { av[cs * 32 + k] = a; bv[cs * 32 + k] = b; };
    const float u24 = ldexpf(1.f, -24), u25 = ldexpf(1.f, -25);
    name[0] = "1 + 2^-24 + 2^-25 (0.75 ulp above 1)";  set(0, 0, 1, 1); set(0, 1, u24, 1); set(0, 2, u25, 1);
    exact[0] = 1.0 + ldexp(1.0, -24) + ldexp(1.0, -25);
    name[1] = "same, small terms first";  set(1, 0, u25, 1); set(1, 1, u24, 1); set(1, 31, 1, 1);
    exact[1] = exact[0];
    name[2] = "C = 1 plus 2^-24 + 2^-25";  c00[2] = 1.0f; set(2, 0, u24, 1); set(2, 1, u25, 1);
    exact[2] = exact[0];
    name[3] = "1 - 1 + 2^-30 (cancellation)";  set(3, 0, 1, 1); set(3, 1, -1, 1); set(3, 2, ldexpf(1.f, -30), 1);
    exact[3] = ldexp(1.0, -30);
    name[4] = "1 + 2^-24 (a tie)";  set(4, 0, 1, 1); set(4, 1, u24, 1);
    exact[4] = 1.0 + ldexp(1.0, -24);
    name[5] = "1 + 2^-24 + 2^-40 (just above a tie)";  set(5, 0, 1, 1); set(5, 1, u24, 1); set(5, 2, ldexpf(1.f, -40), 1);
    exact[5] = 1.0 + ldexp(1.0, -24) + ldexp(1.0, -40);
    name[6] = "-(1 + 2^-24 + 2^-25)";  set(6, 0, -1, 1); set(6, 1, -u24, 1); set(6, 2, -u25, 1);
    exact[6] = -exact[0];
    name[7] = "C = 1 plus 2^-24 + 2^-40";  c00[7] = 1.0f; set(7, 0, u24, 1); set(7, 1, ldexpf(1.f, -40), 1);
    exact[7] = 1.0 + ldexp(1.0, -24) + ldexp(1.0, -40);
    float *da = nullptr, *db = nullptr, *dc = nullptr, *dout = nullptr;
    if (hipMalloc(&da, sizeof(av)) != hipSuccess || hipMalloc(&db, sizeof(bv)) != hipSuccess ||
        hipMalloc(&dc, sizeof(c00)) != hipSuccess || hipMalloc(&dout, NCASE * 256 * sizeof(float)) != hipSuccess ||
        hipMemcpy(da, av, sizeof(av), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(db, bv, sizeof(bv), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dc, c00, sizeof(c00), hipMemcpyHostToDevice) != hipSuccess) {
        printf("set-up failed\n");
        return 1;
    }
    hipLaunchKernelGGL(probe, dim3(NCASE), dim3(64), 0, 0, da, db, dc, dout);
    static float out[NCASE * 256];
    if (hipMemcpy(out, dout, sizeof(out), hipMemcpyDeviceToHost) != hipSuccess) { printf("copy failed\n"); return 1; }
    for (int cs = 0; cs < NCASE; ++cs) {
        const float g = out[cs * 256];
        const float rne = (float)exact[cs];
        unsigned gb, rb; memcpy(&gb, &g, 4); memcpy(&rb, &rne, 4);
        printf("%-40s got %.9g (0x%08x)  RNE %.9g (0x%08x)  exact %.12g  %s\n", name[cs], g, gb, rne, rb, exact[cs],
               gb == rb ? "= RNE" : "differs");
    }
    return 0;
}

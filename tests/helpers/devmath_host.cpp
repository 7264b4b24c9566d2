// Host harness around the kernels' own arithmetic (dev_common.hpp is
// __host__ __device__): reads commands from stdin, prints results, so that the
// tests can compare the code the GPU runs with the CPU oracle without a GPU.
//
//   draw  seed stream j T F L D        -> t0 t2 f0 f1 f2 dtau
//   rows  t0 t2 f0 f1 f2               -> N rows (DDA walk)
//   rowsat t0 t2 f0 f1 f2 k0           -> N rows, DDA started at k0 <= 0 and stepped to 0
//   rowsf t0 t2 f0 f1 f2 k0            -> N rows of the FP64 walk started at k0 <= 0
//   rot   ph pr pi                     -> Re[exp(2 pi i ph/2^32)(pr + i pi)] as %.9e
//   phx   fq4_lo dfq4 dtau row         -> the scorers' phase argument (FP32 turns in [1, 2))
//   key   z j                          -> 64-bit key (hex)
//   drawtm seed stream j T F L D       -> t0 t1 t2 f0 f1 f2 dtau (free t_mid)
//   rowstm t0 t1 t2 f0 f1 f2           -> N rows of a free-t_mid template
//   tmstat t0 t1 t2 f0 f1 f2           -> columns whose FP32 pass fell back to the exact path
//   tmerr t0 t1 t2 f0 f1 f2            -> largest |y32 - y| / tol over the columns (y in FP64)
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "dev_common.hpp"

using namespace stt;

#ifdef STT_HOST_ULP_PERTURB
// One-ulp moves of the square roots and reciprocals of the free-t_mid rows' FP32 pass, in a
// pseudo-random direction: a harsher error than the hardware's (within 1 ulp), so that rows
// staying exact here show the certified window covers the device.
namespace stt {
float stt_host_perturb(float x)
{
    static uint32_t s = 0x9E3779B9u;
    s = s * 1664525u + 1013904223u;
    if (x == 0.0f) return x;
    return std::nextafter(x, (s >> 31) ? INFINITY : -INFINITY);
}
}  // namespace stt
#endif

int main()
{
    char cmd[16];
    while (std::scanf("%15s", cmd) == 1) {
        if (!std::strcmp(cmd, "draw")) {
            unsigned long long seed, j;
            unsigned stream;
            int T, F, L, D;
            if (std::scanf("%llu %u %llu %d %d %d %d", &seed, &stream, &j, &T, &F, &L, &D) != 7) return 2;
            GenP g;
            const long long npos = T - L + 1;
            g.key0 = (uint32_t)seed;
            g.key1 = (uint32_t)(seed >> 32);
            g.stream = stream;
            g.npairs = (uint32_t)(npos * (npos + 1) / 2);
            g.L = L;
            g.frange = (uint32_t)F << 8;
            g.dmax = D;
            g.dspan = 2u * (uint32_t)D + 1u;
            const Trk t = draw_track(g, j);
            int32_t a, b;
            draw_extent(g, j, a, b);
            if (a != t.t0 || b != t.t2) return 3;
            std::printf("%d %d %u %u %u %d\n", t.t0, t.t2, t.f0, t.f1, t.f2, t.dtau);
        } else if (!std::strcmp(cmd, "drawtm")) {
            unsigned long long seed, j;
            unsigned stream;
            int T, F, L, D;
            if (std::scanf("%llu %u %llu %d %d %d %d", &seed, &stream, &j, &T, &F, &L, &D) != 7) return 2;
            GenP g;
            const long long npos = T - L + 1;
            g.key0 = (uint32_t)seed;
            g.key1 = (uint32_t)(seed >> 32);
            g.stream = stream;
            g.npairs = (uint32_t)(npos * (npos + 1) / 2);
            g.L = L;
            g.frange = (uint32_t)F << 8;
            g.dmax = D;
            g.dspan = 2u * (uint32_t)D + 1u;
            const TrkTm t = draw_track_tm(g, j);
            std::printf("%d %d %d %u %u %u %d\n", t.t0, t.t1, t.t2, t.f0, t.f1, t.f2, t.dtau);
        } else if (!std::strcmp(cmd, "rowstm")) {
            TrkTm t;
            if (std::scanf("%d %d %d %u %u %u", &t.t0, &t.t1, &t.t2, &t.f0, &t.f1, &t.f2) != 6) return 2;
            t.dtau = 0;
            const RowTm k = row_tm_init(t);
            for (int dt = 0; dt <= t.t2 - t.t0; ++dt) std::printf(dt ? " %d" : "%d", row_tm(k, dt));
            std::printf("\n");
        } else if (!std::strcmp(cmd, "tmstat")) {
            TrkTm t;
            if (std::scanf("%d %d %d %u %u %u", &t.t0, &t.t1, &t.t2, &t.f0, &t.f1, &t.f2) != 6) return 2;
            t.dtau = 0;
            const RowTm k = row_tm_init(t);
            int nfb = 0;
            for (int dt = 1; dt <= t.t2 - t.t0; ++dt) {
                bool ok;
                (void)row_tm_fp32(k, dt, ok);
                nfb += !ok;
            }
            std::printf("%d %.6e\n", nfb, (double)k.tol);
        } else if (!std::strcmp(cmd, "tmerr")) {
            TrkTm t;
            if (std::scanf("%d %d %d %u %u %u", &t.t0, &t.t1, &t.t2, &t.f0, &t.f1, &t.f2) != 6) return 2;
            t.dtau = 0;
            const RowTm k = row_tm_init(t);
            const double b = 2.0 * (t.t1 - t.t0);
            const double B = 2.0 * ((double)t.f1 - t.f0), C = (double)t.f0 - 2.0 * t.f1 + t.f2;
            double worst = 0.0;
            for (int dt = 1; dt <= t.t2 - t.t0; ++dt) {
                const int32_t D = k.bb + k.a4 * dt;
                const float xi32 = (float)(2 * dt) * rcp_1ulp(k.bf + sqrt_1ulp((float)D));
                const float y32 = fmaf(xi32, fmaf(xi32, k.Cs, k.Bs), k.fs);
                const double xi = 2.0 * dt / (b + std::sqrt((double)D));
                const double y = (t.f0 + xi * (B + C * xi)) / 256.0;
                worst = std::fmax(worst, std::fabs((double)y32 - y) / (double)k.tol);
            }
            std::printf("%.6f\n", worst);
        } else if (!std::strcmp(cmd, "rows")) {
            Trk t;
            if (std::scanf("%d %d %u %u %u", &t.t0, &t.t2, &t.f0, &t.f1, &t.f2) != 5) return 2;
            t.dtau = 0;
            Dda s = dda_init(t);
            const int N = t.t2 - t.t0 + 1;
            for (int k = 0; k < N; ++k) {
                std::printf(k ? " %d" : "%d", s.row);
                dda_step(s);
            }
            std::printf("\n");
        } else if (!std::strcmp(cmd, "rowsat")) {  // rows from a rewound start k0 <= 0
            Trk t;
            int k0;
            if (std::scanf("%d %d %u %u %u %d", &t.t0, &t.t2, &t.f0, &t.f1, &t.f2, &k0) != 6) return 2;
            t.dtau = 0;
            Dda s = dda_init_at(t, k0);
            for (int k = k0; k < 0; ++k) dda_step(s);
            const int N = t.t2 - t.t0 + 1;
            for (int k = 0; k < N; ++k) {
                std::printf(k ? " %d" : "%d", s.row);
                dda_step(s);
            }
            std::printf("\n");
        } else if (!std::strcmp(cmd, "rowsf")) {  // FP64 walk from k0 <= 0
            Trk t;
            int k0;
            if (std::scanf("%d %d %u %u %u %d", &t.t0, &t.t2, &t.f0, &t.f1, &t.f2, &k0) != 6) return 2;
            t.dtau = 0;
            DdaF s = ddaf_init_at(t, k0);
            for (int k = k0; k < 0; ++k) ddaf_step(s);
            const int N = t.t2 - t.t0 + 1;
            for (int k = 0; k < N; ++k) {
                std::printf(k ? " %d" : "%d", ddaf_row(s));
                ddaf_step(s);
            }
            std::printf("\n");
        } else if (!std::strcmp(cmd, "rot")) {
            unsigned ph;
            float pr, pi;
            if (std::scanf("%u %f %f", &ph, &pr, &pi) != 3) return 2;
            std::printf("%.9e\n", (double)rot_re(ph, pr, pi));
        } else if (!std::strcmp(cmd, "phx")) {  // the scorers' FP32 phase argument, in turns
            int fq4_lo, dfq4, dtau, row;
            if (std::scanf("%d %d %d %d", &fq4_lo, &dfq4, &dtau, &row) != 4) return 2;
            std::printf("%.9e\n", (double)phase_turns(phase_a(fq4_lo, dtau), phase_b(dfq4, dtau), row));
        } else if (!std::strcmp(cmd, "key")) {
            float z;
            unsigned j;
            if (std::scanf("%f %u", &z, &j) != 2) return 2;
            std::printf("%016llx\n", (unsigned long long)key_encode(z, j));
        } else {
            return 1;
        }
        std::fflush(stdout);
    }
    return 0;
}

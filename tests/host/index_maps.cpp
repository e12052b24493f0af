// Host-side checks of the index maps the hopping kernels use (compiled for the
// host only; the same __host__ __device__ functions run in the kernels):
//  * fdiv (division by an invariant divisor, multiply-high and shifts) equals
//    integer division for every divisor the z-range processing order produces
//    (chunk sites k Lt (Lx/2) Ly and plane sites k (Lx/2) Ly) and every position;
//  * yz_site (the y-z block order) is a bijection of [0, Vh) that keeps block b
//    inside y in [(b % 2) Ly/2, +Ly/2) and z in [(b / 2) Lz/4, +Lz/4).
// Prints "ok" and exits 0, or prints the first failure and exits 1.
#include <cstdio>
#include <vector>

#include "wl_dslash.h"

using namespace wl;

static Geom geom(const int d[4]) {
    Geom g{};
    for (int m = 0; m < 4; ++m) g.L[m] = d[m];
    g.lxh = d[0] / 2;
    g.vh = g.lxh * d[1] * d[2] * d[3];
    g.sy = g.lxh;
    g.sz = g.lxh * d[1];
    g.st = g.sz * d[2];
    g.f_lxh = make_fastdiv(g.lxh);
    g.f_ly = make_fastdiv(d[1]);
    g.f_lz = make_fastdiv(d[2]);
    g.f_sz = make_fastdiv(g.sz);
    return g;
}

int main() {
    const int shapes[][4] = {{24, 24, 24, 48}, {32, 32, 32, 64}, {16, 16, 16, 32}, {8, 8, 8, 8}, {12, 12, 12, 24},
                             {4, 4, 4, 4},     {8, 2, 4, 6},     {6, 6, 8, 10},    {20, 22, 12, 14}, {2, 2, 4, 2}};
    for (const auto &d : shapes) {
        const Geom g = geom(d);
        // z-range divisors
        for (int k = 1; k < d[2]; ++k) {
            const int divs[2] = {k * d[3] * g.sz, k * g.sz};
            for (int dv : divs) {
                const FastDiv f = make_fastdiv(dv);
                for (int n = 0; n < g.vh; ++n)
                    if (fdiv(n, f) != n / dv) {
                        printf("fdiv(%d, %d) = %d, expected %d\n", n, dv, fdiv(n, f), n / dv);
                        return 1;
                    }
            }
        }
        // y-z blocks
        if (d[1] % 2 || d[2] % 4) continue;
        const int by = d[1] / 2, bz = d[2] / 4;
        const FastDiv f_row = make_fastdiv(by * g.lxh), f_slab = make_fastdiv(bz * by * g.lxh),
                      f_blk = make_fastdiv(d[3] * bz * by * g.lxh);
        std::vector<int> seen(g.vh, 0);
        const int per_blk = g.vh / 8;
        for (int ps = 0; ps < g.vh; ++ps) {
            const int i = yz_site(g, by, bz, f_blk, f_slab, f_row, ps);
            if (i < 0 || i >= g.vh || seen[i]++) {
                printf("%dx%dx%dx%d: position %d -> site %d (out of range or repeated)\n", d[0], d[1], d[2], d[3], ps, i);
                return 1;
            }
            const int y = (i / g.lxh) % d[1], z = (i / g.sz) % d[2], b = ps / per_blk;
            if (y / by != (b & 1) || z / bz != (b >> 1)) {
                printf("%dx%dx%dx%d: position %d (block %d) -> y %d z %d\n", d[0], d[1], d[2], d[3], ps, b, y, z);
                return 1;
            }
        }
    }
    printf("ok\n");
    return 0;
}

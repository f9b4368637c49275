// Host-side reference for the Philox4x32-10 pin: calls rocRAND's own
// philox4x32_10 engine (the installed library header) on the host.
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin, prints "r0 r1 r2 r3" (hex).
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

// ten_rounds is a protected member of the engine; a subclass re-exports it.
struct philox_rounds : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    philox_rounds eng;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = eng.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}

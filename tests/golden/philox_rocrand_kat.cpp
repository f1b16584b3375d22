// Test-only known-answer generator: evaluates the Philox4x32-10 block function
// of AMD's MIT-licensed rocRAND header (an implementation independent of this
// repository's two) on counter/key pairs read from stdin, one per line:
//   c0 c1 c2 c3 k0 k1   (hex)   ->   o0 o1 o2 o3 (hex)
// Never linked into the product library or the oracle.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct kat_engine : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    kat_engine e;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 o = e.block(make_uint4(c0, c1, c2, c3), make_uint2(k0, k1));
        std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}

// Data-consistency kernel instances for nz = 14 (the 256x256x14 cardiac geometry): radix 14
// = 2 x 7 along z, so 28 points per thread and power-of-two ny.
#include "pls_dc_impl.hpp"

namespace pls {

int dc_launch_nz14(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s) {
    switch (ny) {
        case 16: return dc_launch_t<16, 14>(a, bt, s);
        case 32: return dc_launch_t<32, 14>(a, bt, s);
        case 64: return dc_launch_t<64, 14>(a, bt, s);
        case 128: return dc_launch_t<128, 14>(a, bt, s);
        case 256: return dc_launch_t<256, 14>(a, bt, s);
    }
    return -1;
}

}  // namespace pls

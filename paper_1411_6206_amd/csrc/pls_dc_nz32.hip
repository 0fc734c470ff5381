// Data-consistency kernel instances for nz = 32.
#include "pls_dc_impl.hpp"

namespace pls {

int dc_launch_nz32(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s) {
    switch (ny) {
        case 16: return dc_launch_t<16, 32>(a, bt, s);
        case 24: return dc_launch_t<24, 32>(a, bt, s);
        case 32: return dc_launch_t<32, 32>(a, bt, s);
        case 48: return dc_launch_t<48, 32>(a, bt, s);
        case 64: return dc_launch_t<64, 32>(a, bt, s);
        case 96: return dc_launch_t<96, 32>(a, bt, s);
        case 128: return dc_launch_t<128, 32>(a, bt, s);
        case 192: return dc_launch_t<192, 32>(a, bt, s);
        case 256: return dc_launch_t<256, 32>(a, bt, s);
    }
    return -1;
}

}  // namespace pls

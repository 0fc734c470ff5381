// Data-consistency kernel instances for nz = 16.
#include "pls_dc_impl.hpp"

namespace pls {

int dc_launch_nz16(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s) {
    switch (ny) {
        case 16: return dc_launch_t<16, 16>(a, bt, s);
        case 24: return dc_launch_t<24, 16>(a, bt, s);
        case 32: return dc_launch_t<32, 16>(a, bt, s);
        case 48: return dc_launch_t<48, 16>(a, bt, s);
        case 64: return dc_launch_t<64, 16>(a, bt, s);
        case 96: return dc_launch_t<96, 16>(a, bt, s);
        case 128: return dc_launch_t<128, 16>(a, bt, s);
        case 192: return dc_launch_t<192, 16>(a, bt, s);
        case 256: return dc_launch_t<256, 16>(a, bt, s);
    }
    return -1;
}

}  // namespace pls

// Data-consistency kernel instances for nz = 4.
#include "pls_dc_impl.hpp"

namespace pls {

int dc_launch_nz4(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s) {
    switch (ny) {
        case 16: return dc_launch_t<16, 4>(a, bt, s);
        case 24: return dc_launch_t<24, 4>(a, bt, s);
        case 32: return dc_launch_t<32, 4>(a, bt, s);
        case 48: return dc_launch_t<48, 4>(a, bt, s);
        case 64: return dc_launch_t<64, 4>(a, bt, s);
        case 96: return dc_launch_t<96, 4>(a, bt, s);
        case 128: return dc_launch_t<128, 4>(a, bt, s);
        case 192: return dc_launch_t<192, 4>(a, bt, s);
        case 256: return dc_launch_t<256, 4>(a, bt, s);
    }
    return -1;
}

}  // namespace pls

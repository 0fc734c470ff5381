// Data-consistency kernel instances for nz = 1.
#include "pls_dc_impl.hpp"

namespace pls {

int dc_launch_nz1(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s) {
    switch (ny) {
        case 16: return dc_launch_t<16, 1>(a, bt, s);
        case 24: return dc_launch_t<24, 1>(a, bt, s);
        case 32: return dc_launch_t<32, 1>(a, bt, s);
        case 48: return dc_launch_t<48, 1>(a, bt, s);
        case 64: return dc_launch_t<64, 1>(a, bt, s);
        case 96: return dc_launch_t<96, 1>(a, bt, s);
        case 128: return dc_launch_t<128, 1>(a, bt, s);
        case 192: return dc_launch_t<192, 1>(a, bt, s);
        case 256: return dc_launch_t<256, 1>(a, bt, s);
    }
    return -1;
}

bool xifft_launch_any(int nx, const XiArgs& a, hipStream_t s) {
    switch (nx) {
        case 16: xifft_launch_t<16>(a, s); return true;
        case 24: xifft_launch_t<24>(a, s); return true;
        case 32: xifft_launch_t<32>(a, s); return true;
        case 48: xifft_launch_t<48>(a, s); return true;
        case 64: xifft_launch_t<64>(a, s); return true;
        case 96: xifft_launch_t<96>(a, s); return true;
        case 128: xifft_launch_t<128>(a, s); return true;
        case 192: xifft_launch_t<192>(a, s); return true;
        case 256: xifft_launch_t<256>(a, s); return true;
    }
    return false;
}

}  // namespace pls

// Shape dispatch of the data-consistency pass and the set-up kx inverse DFT.
#include "pls_dc_impl.hpp"

namespace pls {

static const int kNY[] = {16, 24, 32, 48, 64, 96, 128, 192, 256};
static const int kNZ[] = {1, 4, 8, 16, 32};

static bool in_list(int v, const int* l, int n) {
    for (int i = 0; i < n; ++i)
        if (l[i] == v) return true;
    return false;
}

static const int kNY14[] = {16, 32, 64, 128, 256};   // nz = 14 needs 7 | Q: powers of two in y

bool dc_supported(int ny, int nz) {
    if (nz == 14) return in_list(ny, kNY14, 5);
    return in_list(ny, kNY, 9) && in_list(nz, kNZ, 5);
}

bool xifft_supported(int nx) { return in_list(nx, kNY, 9); }

template <int NZ>
static int grid_for(int ny, int nx, int nt) {
    switch (ny) {
        case 16: return dc_grid<16, NZ>(nx, nt);
        case 24: return dc_grid<24, NZ>(nx, nt);
        case 32: return dc_grid<32, NZ>(nx, nt);
        case 48: return dc_grid<48, NZ>(nx, nt);
        case 64: return dc_grid<64, NZ>(nx, nt);
        case 96: return dc_grid<96, NZ>(nx, nt);
        case 128: return dc_grid<128, NZ>(nx, nt);
        case 192: return dc_grid<192, NZ>(nx, nt);
        case 256: return dc_grid<256, NZ>(nx, nt);
    }
    return 0;
}

static int grid_for14(int ny, int nx, int nt) {
    switch (ny) {
        case 16: return dc_grid<16, 14>(nx, nt);
        case 32: return dc_grid<32, 14>(nx, nt);
        case 64: return dc_grid<64, 14>(nx, nt);
        case 128: return dc_grid<128, 14>(nx, nt);
        case 256: return dc_grid<256, 14>(nx, nt);
    }
    return 0;
}

int dc_blocks(int ny, int nz, int nx, int nt) {
    switch (nz) {
        case 1: return grid_for<1>(ny, nx, nt);
        case 4: return grid_for<4>(ny, nx, nt);
        case 8: return grid_for<8>(ny, nx, nt);
        case 14: return grid_for14(ny, nx, nt);
        case 16: return grid_for<16>(ny, nx, nt);
        case 32: return grid_for<32>(ny, nx, nt);
    }
    return 0;
}

int launch_dc_batched(int ny, int nz, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s) {
    int r = -1;
    switch (nz) {
        case 1: r = dc_launch_nz1(ny, a, bt, s); break;
        case 4: r = dc_launch_nz4(ny, a, bt, s); break;
        case 8: r = dc_launch_nz8(ny, a, bt, s); break;
        case 14: r = dc_launch_nz14(ny, a, bt, s); break;
        case 16: r = dc_launch_nz16(ny, a, bt, s); break;
        case 32: r = dc_launch_nz32(ny, a, bt, s); break;
    }
    return r < 0 ? 0 : r;
}

int launch_dc(int ny, int nz, const DcArgs& a, hipStream_t s) {
    return launch_dc_batched(ny, nz, a, nullptr, s);
}

bool launch_xifft(int nx, const XiArgs& a, hipStream_t s) { return xifft_launch_any(nx, a, s); }

}  // namespace pls

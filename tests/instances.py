"""The kernel instances the header (include/prior_ls.h, prior_ls_dims) advertises: one
data-consistency kernel per (ny, nz) phase-encode plane, one kx inverse DFT per readout
length nx."""
PLANE_NY = (16, 24, 32, 48, 64, 96, 128, 192, 256)
PLANE_NZ = (1, 4, 8, 16, 32)
PLANE_NY_NZ14 = (16, 32, 64, 128, 256)      # nz = 14: radix 14 = 2 x 7 along z
READOUT_NX = (16, 24, 32, 48, 64, 96, 128, 192, 256)

PLANES = [(ny, nz) for nz in PLANE_NZ for ny in PLANE_NY] + [(ny, 14) for ny in PLANE_NY_NZ14]

"""Mixed-precision Paterson--Stockmeyer evaluation of matrix polynomials on
AMD MI355X (gfx950).  The compute path is the C-ABI library libps.so built
from csrc/ (hand-written HIP kernels); this package only marshals arguments.
Importing the package does not load the library; the first call does, and it
raises if the library is missing."""

"""MI355X (gfx950) library for the SAP-preconditioned aggregation multilevel
solver of the Wilson-clover Dirac equation (Frommer, Kahl, Krieg, Leder,
Rottmann, Lattice 2011). The compute path is libmgdd.so (hand-written HIP);
`paper_1202_2462_amd.mgdd` is its ctypes binding."""

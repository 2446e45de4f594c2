"""MI355X-native MPDATA time step (libmpdata++ 0.1, Sect. 3.1) behind a C ABI.

The compute path is the HIP library libmpdata.so (paper_1407_1309_amd/csrc);
`paper_1407_1309_amd.mpdata` is its thin ctypes binding.  Importing this
package loads nothing; the binding loads the library on first use and raises
if it is missing.
"""

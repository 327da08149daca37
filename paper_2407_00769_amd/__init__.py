"""tnc: sliced tensor-network amplitudes on one MI355X (gfx950).

The compute path is the HIP library ``libtnc.so`` behind a C ABI
(``include/tnc.h``); ``paper_2407_00769_amd._tnc`` binds it with ctypes and
``circuit_network`` marshals circuits into its tensor-list input.
"""

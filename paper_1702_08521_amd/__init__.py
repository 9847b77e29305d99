"""MI355X-native SL-MPP5/7 Vlasov advection sweeps (arXiv:1702.08521).

The compute path is the HIP library ``libslmpp.so`` built from ``csrc/``;
``slmpp`` is its thin ctypes binding.  ``workloads`` generates seeded
synthetic inputs.
"""
__all__ = ["slmpp", "workloads"]

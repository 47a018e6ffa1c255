"""MI355X-native ANI-style neural-network-potential energy and forces.

The GPU library (`libnnp_hip.so`, HIP for gfx950) is loaded lazily by
`paper_2201_08110_amd.nnp`; importing the package itself touches no GPU and
loads no native code, so the seeded input generators in
`paper_2201_08110_amd.synth` can be used on machines without one.
"""

__all__ = ["synth"]

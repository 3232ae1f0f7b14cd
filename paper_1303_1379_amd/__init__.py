"""MI355X-native maximum-cardinality bipartite matching (APFB with GPUBFS-WR,
Alternate and FixMatching) behind a C ABI (``libmcm.so``)."""

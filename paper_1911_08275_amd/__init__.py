"""MI355X-native gridded pair counting (cell lists, bounding-box pruned cell
pairs, FP32 distances with an FP64 edge recheck) for xi(r) and wp(rp)."""
__all__ = ["synth"]

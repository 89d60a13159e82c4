"""MI355X-native extension + volume FMM (Fryklund & Greengard, function
extension from cut leaves followed by an adaptive volume FMM).

    from paper_2211_14537_amd import vfx, tree
"""

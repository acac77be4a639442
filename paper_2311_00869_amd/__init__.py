"""MI355X-native graphBpp spanning-tree sweep and graphL (see ``frustration``)."""
